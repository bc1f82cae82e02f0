// Ab initio deflection angle by quadrature of the classical deflection
// integral (section "Computational Implementation: The Exact vs. Neural
// Paradigm"): the batch entry point, Phase A of the in-step rule, the
// training-row harvest and the Chapman-Enskog transport integrals.  The
// per-pair arithmetic (root, substitution, Gauss-Legendre rule, peak
// detection and the FP64 refinement pieces) is in chi_quad.hpp; this file
// holds the wave-level driver -- every lane evaluates its pair, then the
// wavefront re-evaluates each flagged pair in FP64 together -- and the
// kernels.
#include <math.h>

#include <string.h>

#include <vector>

#include "chi_quad.hpp"
#include "collide.hpp"

namespace dsmc {

// ------------------------------------------------------------------------
// Wave level: the lane rule for every pair, then the FP64 refinement of the
// flagged pairs, one pair at a time by the whole wavefront.
// ------------------------------------------------------------------------
// chi of one pair re-evaluated in FP64 by the 64 lanes of a wave (all lanes
// call it with the same b, E), with uniform control flow:
//  1. D at 64 geometric radii (one per lane) from max(b, r_zero) down past
//     r_floor; the first sign change bounds the largest root from below.
//  2. If the samples show a local minimum of D above it, D' is bracketed
//     there by parallel rounds: a minimum D(r_m) <= 0 means a dip holding
//     the largest root in (r_m, r_{k-1}); a positive one is the interior
//     peak of the integrand.
//  3. The root is bracketed by parallel rounds, the secant taken, and V, V'
//     evaluated there; D'' at r_min by a central difference on two lanes.
//  4. The sinh-mapped integral, its nodes spread over the lanes, summed by a
//     fixed butterfly.
__device__ double chi_refine_wave(const Pot& P, const QuadCfg& q, const GLRule& gl, double b,
                                  double E)
{
    const int lane = threadIdx.x & 63;
    RefState s{};
    s.b2 = b * b;
    s.E = E;
    double rtop, rho;
    ref_grid(P, b, rtop, rho);
    const double r = ref_sample_r(rtop, rho, lane);
    const double D = D_of<double>(P, s.b2, E, r);
    const double Dup = __shfl(D, lane > 0 ? lane - 1 : 0, 64);
    const double Ddn = __shfl(D, lane < 63 ? lane + 1 : 63, 64);
    const uint64_t neg = __ballot(D <= 0.0);
    if (!neg) return NAN;
    const int kneg = __ffsll((unsigned long long)neg) - 1;
    double rlo = __shfl(r, kneg, 64);
    double rhi = __shfl(r, kneg > 0 ? kneg - 1 : 0, 64);
    const uint64_t mins = __ballot(lane >= 1 && lane < kneg && D < Dup && D < Ddn);
    bool has_min = false;
    double rm = 0.0, dm = 0.0, d2m = 0.0;
    if (mins) {
        const int k = __ffsll((unsigned long long)mins) - 1;
        double a = __shfl(r, k + 1, 64), bb = __shfl(r, k - 1, 64), fa = 0.0, fb = 0.0;
        for (int rd = 0; rd < REF_ROUNDS; ++rd) {
            const double x = ref_x(a, bb, lane);
            const double f = dD_of<double>(P, s.b2, E, x);
            const uint64_t pos = __ballot(f >= 0.0);
            const int L = ref_pick(pos ? __ffsll((unsigned long long)pos) - 1 : 64);
            a = __shfl(x, L - 1, 64);
            bb = __shfl(x, L, 64);
            fa = __shfl(f, L - 1, 64);
            fb = __shfl(f, L, 64);
        }
        rm = (fb > fa) ? a - fa * (bb - a) / (fb - fa) : 0.5 * (a + bb);
        rm = fmin(fmax(rm, a), bb);
        d2m = (fb - fa) / (bb - a);
        dm = D_of<double>(P, s.b2, E, rm);
        if (dm <= 0.0) {
            // the dip reaches zero: the largest root lies in (r_m, r_{k-1})
            rlo = rm;
            rhi = __shfl(r, k - 1, 64);
        } else {
            has_min = true;
        }
    }
    // root of D in [rlo, rhi] (D(rlo) <= 0 < D(rhi); equal ends if D(rtop) <= 0)
    double fl = -1.0, fh = 1.0;
    for (int rd = 0; rd < REF_ROUNDS && rhi > rlo; ++rd) {
        const double x = ref_x(rlo, rhi, lane);
        const double f = D_of<double>(P, s.b2, E, x);
        const uint64_t pos = __ballot(f > 0.0);
        const int L = ref_pick(pos ? __ffsll((unsigned long long)pos) - 1 : 64);
        rlo = __shfl(x, L - 1, 64);
        rhi = __shfl(x, L, 64);
        fl = __shfl(f, L - 1, 64);
        fh = __shfl(f, L, 64);
    }
    s.rmin = (rhi > rlo && fh > fl) ? rlo - fl * (rhi - rlo) / (fh - fl) : rlo;
    s.rmin = fmin(fmax(s.rmin, rlo), rhi);
    double dV;
    s.Vmin = pot_eval<double, true>(P, s.rmin, dV);
    const double dD = 2.0 * s.b2 / (s.rmin * s.rmin * s.rmin) - dV / E;
    s.beta = b / s.rmin;
    // D''(r_min) by a central difference, one side on each of two lanes
    const double h = 1e-4 * s.rmin;
    const double fd = dD_of<double>(P, s.b2, E, s.rmin + (lane == 0 ? h : -h));
    const double d2D = (__shfl(fd, 0, 64) - __shfl(fd, 1, 64)) / (2.0 * h);
    ref_map(s, has_min, rm, dm, d2m, dD, d2D);
    const int M = ref_nodes(s, gl);
    double I = 0.0;
    int nonpos = 0;
    for (int m = lane; m < M; m += 64) I += ref_node(P, gl, s, m, nonpos);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) I += __shfl_xor(I, o, 64);
    return 3.14159265358979323846 - 2.0 * s.beta * I;
}

// chi for the lanes of a wave with the refinement done in place (all 64
// lanes call it; inactive lanes pass active = false).  Used where the items
// are not stored in a form a separate pass could re-read (the transport
// integrals' b nodes); FP64 only.
__device__ double chi_wave_inplace(const Pot& P, const QuadCfg& q, const GLRule& gl, double b,
                                   double E, bool active)
{
    bool flag = false;
    double c = 0.0;
    if (active) c = chi_lane<double>(P, q, gl, b, E, flag);
    if (!q.refine) return c;
    uint64_t pend = __ballot(active && flag);
    const int lane = threadIdx.x & 63;
    while (pend) {
        const int src = __ffsll((unsigned long long)pend) - 1;
        const double cr = chi_refine_wave(P, q, gl, __shfl(b, src, 64), __shfl(E, src, 64));
        if (lane == src) c = cr;
        pend &= pend - 1;
    }
    return c;
}

// Refinement pass: each wave scans 64 consecutive items, and every item the
// lane pass left pending (a sentinel in its output) is re-evaluated by the
// whole wave.  Job supplies count(n) (the items to scan, at most n),
// pending(i), inputs(i, b, E) and store(i, chi).
template <class Job>
__global__ void __launch_bounds__(256)
k_refine(Job job, int64_t n, Pot P, QuadCfg q, GLRule gl, dsmc_status* st)
{
    n = job.count(n);
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t base = wave * 64; base < n; base += n_waves * 64) {
        const int64_t i = base + lane;
        uint64_t pend = __ballot(i < n && job.pending(i));
        while (pend) {
            const int src = __ffsll((unsigned long long)pend) - 1;
            double b = 0.0, E = 0.0;
            if (lane == src) job.inputs(i, b, E);
            b = __shfl(b, src, 64);
            E = __shfl(E, src, 64);
            const double c = chi_refine_wave(P, q, gl, b, E);
            if (lane == src) {
                if (c != c && st) {
                    atomicAdd(&st->root_fail, 1);
                    atomicOr(&st->flags, (uint32_t)DSMC_ST_ROOT_FAIL);
                }
                job.store(i, c);
            }
            pend &= pend - 1;
        }
    }
}

// Sentinel of a pending item: +inf (no chi, cos chi or integrand term takes it).
template <typename T> __device__ __forceinline__ T pending_mark() { return T(INFINITY); }
template <typename T> __device__ __forceinline__ bool is_pending(T x) { return x == T(INFINITY); }

// Host-side potential set-up is costly for JAGER (grid search); cache the
// last one.
static bool same_pot(const dsmc_potential& a, const dsmc_potential& b)
{
    return memcmp(&a, &b, sizeof(a)) == 0;
}

static int get_pot(const dsmc_potential* pot, Pot* out)
{
    static thread_local bool have = false;
    static thread_local Pot cached;
    if (have && pot && same_pot(cached.p, *pot)) {
        *out = cached;
        return DSMC_OK;
    }
    int rc = make_pot(pot, out);
    if (rc == DSMC_OK) {
        cached = *out;
        have = true;
    }
    return rc;
}

constexpr double KB = 1.380649e-23;

__device__ __forceinline__ void count_root_fail(dsmc_status* st)
{
    if (st) {
        atomicAdd(&st->root_fail, 1);
        atomicOr(&st->flags, (uint32_t)DSMC_ST_ROOT_FAIL);
    }
}

// ------------------------------------------------------------------------
// Kernels.  Each lane-pass kernel evaluates its items with the lane rule and
// leaves the flagged ones pending; k_refine with the matching job finishes
// them.
// ------------------------------------------------------------------------
// Lane pass of the batch entry point.
template <typename T>
__device__ __forceinline__ void deflect_lanes(int64_t n, const T* __restrict__ b,
                                              const T* __restrict__ g, T* __restrict__ chi,
                                              double half_m_over_k, const Pot& P, const QuadCfg& q,
                                              const GLRule& gl, int fold, dsmc_status* st)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const double gg = double(g[p]);
        bool flag;
        T c = chi_lane<T>(P, q, gl, double(b[p]) * 1e10, half_m_over_k * gg * gg, flag);
        if (flag && q.refine) {
            chi[p] = pending_mark<T>();
            continue;
        }
        if (c != c) count_root_fail(st);
        else if (fold) c = acos(cos(c));
        chi[p] = c;
    }
}

// The FP32 lane rule fits in 128 VGPRs: four waves per SIMD instead of three
// hide more of its latency.  The FP64 one would spill under that cap.
__global__ void __launch_bounds__(256)
k_deflect_f64(int64_t n, const double* __restrict__ b, const double* __restrict__ g,
              double* __restrict__ chi, double half_m_over_k, Pot P, QuadCfg q, GLRule gl, int fold,
              dsmc_status* st)
{
    deflect_lanes<double>(n, b, g, chi, half_m_over_k, P, q, gl, fold, st);
}
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_deflect_f32(int64_t n, const float* __restrict__ b, const float* __restrict__ g,
              float* __restrict__ chi, double half_m_over_k, Pot P, QuadCfg q, GLRule gl, int fold,
              dsmc_status* st)
{
    deflect_lanes<float>(n, b, g, chi, half_m_over_k, P, q, gl, fold, st);
}

template <typename T>
struct DeflectJob {
    const T* b;
    const T* g;
    T* chi;
    double half_m_over_k;
    int fold;
    __device__ int64_t count(int64_t n) const { return n; }
    __device__ bool pending(int64_t p) const { return is_pending(chi[p]); }
    __device__ void inputs(int64_t p, double& bb, double& E) const
    {
        const double gg = double(g[p]);
        bb = double(b[p]) * 1e10;
        E = half_m_over_k * gg * gg;
    }
    __device__ void store(int64_t p, double c) const
    {
        chi[p] = T(fold && c == c ? acos(cos(c)) : c);
    }
};

// Impact parameter (Angstrom) and E/k_B of accepted pair p, in FP64 from the
// stored velocities and the pair's latent U4 (b^2 / b_max^2 = 1 - exp(-|z|^2/2) = U4).
template <typename T>
__device__ __forceinline__ void pair_b_E(const PairsView& pr, const dsmc_rng& rng, const V3<const T>& v,
                                         double half_m_over_k, double b_max_A, int64_t p,
                                         T (&xi)[3], double& bb, double& E)
{
    T z[2], u4;
    const int32_t k = pr.cell[p];
    const uint32_t a = (uint32_t)(p - pr.off[k]);
    pair_latents(rng, a, (uint32_t)k, xi, z, u4);
    const int32_t i = pr.i[p], j = pr.j[p];
    const double rx = double(v.x[i]) - double(v.x[j]);
    const double ry = double(v.y[i]) - double(v.y[j]);
    const double rz = double(v.z[i]) - double(v.z[j]);
    E = half_m_over_k * (rx * rx + ry * ry + rz * rz);
    bb = b_max_A * sqrt(double(u4));
}

// Phase A of the in-step ab initio rule.
template <typename T>
__device__ __forceinline__ void phaseA_jager_lanes(int32_t n_cells, const PairsView& pr,
                                                   const dsmc_rng& rng, const V3<const T>& v,
                                                   double half_m_over_k, double b_max_A,
                                                   const Pot& P, const QuadCfg& q, const GLRule& gl,
                                                   const PairBuf<T>& out, dsmc_status* st)
{
    const int64_t np = pr.total(n_cells);
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np;
         p += (int64_t)gridDim.x * blockDim.x) {
        T xi[3];
        double bb, E;
        pair_b_E<T>(pr, rng, v, half_m_over_k, b_max_A, p, xi, bb, E);
        bool flag;
        T c = chi_lane<T>(P, q, gl, bb, E, flag);
        out.c[p] = xi[0];
        out.d[p] = xi[1];
        out.e[p] = xi[2];
        if (flag && q.refine) {
            out.a[p] = pending_mark<T>();
            continue;
        }
        if (c != c) {
            count_root_fail(st);
            c = T(0);  // no deflection for a failed evaluation
        }
        out.a[p] = cos(c);
        out.b[p] = sin(c);
    }
}

__global__ void __launch_bounds__(256)
k_phaseA_jager_f64(int32_t n_cells, PairsView pr, dsmc_rng rng, V3<const double> v,
                   double half_m_over_k, double b_max_A, Pot P, QuadCfg q, GLRule gl,
                   PairBuf<double> out, dsmc_status* st)
{
    phaseA_jager_lanes<double>(n_cells, pr, rng, v, half_m_over_k, b_max_A, P, q, gl, out, st);
}
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_phaseA_jager_f32(int32_t n_cells, PairsView pr, dsmc_rng rng, V3<const float> v,
                   double half_m_over_k, double b_max_A, Pot P, QuadCfg q, GLRule gl,
                   PairBuf<float> out, dsmc_status* st)
{
    phaseA_jager_lanes<float>(n_cells, pr, rng, v, half_m_over_k, b_max_A, P, q, gl, out, st);
}

template <typename T>
struct PhaseAJagerJob {
    PairsView pr;
    dsmc_rng rng;
    V3<const T> v;
    double half_m_over_k, b_max_A;
    PairBuf<T> out;
    int32_t n_cells;
    __device__ int64_t count(int64_t n) const
    {
        const int64_t np = pr.total(n_cells);
        return np < n ? np : n;
    }
    __device__ bool pending(int64_t p) const { return is_pending(out.a[p]); }
    __device__ void inputs(int64_t p, double& bb, double& E) const
    {
        T xi[3];
        pair_b_E<T>(pr, rng, v, half_m_over_k, b_max_A, p, xi, bb, E);
    }
    __device__ void store(int64_t p, double c) const
    {
        if (c != c) c = 0.0;
        out.a[p] = T(cos(c));
        out.b[p] = T(sin(c));
    }
};

// Harvest rows: targets from the quadrature.
__device__ __forceinline__ void harvest_target(const double* vr, const double* xi, int64_t r,
                                               double c, float* tgt, double* chi_out)
{
    double vh[3], e[3];
    const double g = unit3<double>(vr[3 * r], vr[3 * r + 1], vr[3 * r + 2], vh);
    const double xv[3] = {xi[3 * r], xi[3 * r + 1], xi[3 * r + 2]};
    perp_dir<double>(xv, vh, e);
    const double cc = cos(c), sc = sin(c);
    for (int d = 0; d < 3; ++d) tgt[3 * r + d] = (float)(g * (cc * vh[d] + sc * e[d]));
    if (chi_out) chi_out[r] = c;
}

__device__ __forceinline__ void harvest_b_E(const double* vr, const double* z, double b_max_A,
                                            double half_m_over_k, int64_t r, double& bb, double& E)
{
    const double v0 = vr[3 * r], v1 = vr[3 * r + 1], v2 = vr[3 * r + 2];
    const double z0 = z[2 * r], z1 = z[2 * r + 1];
    const double bt2 = -expm1(-0.5 * (z0 * z0 + z1 * z1));
    bb = b_max_A * sqrt(bt2);
    E = half_m_over_k * (v0 * v0 + v1 * v1 + v2 * v2);
}

__global__ void __launch_bounds__(256)
k_harvest(int64_t B, const double* __restrict__ vr, const double* __restrict__ xi,
          const double* __restrict__ z, double inv_sv, double b_max_A, double half_m_over_k,
          Pot P, QuadCfg q, GLRule gl, float* __restrict__ x_out, float* __restrict__ g_out,
          float* __restrict__ tgt, double* __restrict__ chi_out, dsmc_status* st)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < B;
         r += (int64_t)gridDim.x * blockDim.x) {
        const double v0 = vr[3 * r], v1 = vr[3 * r + 1], v2 = vr[3 * r + 2];
        double bb, E;
        harvest_b_E(vr, z, b_max_A, half_m_over_k, r, bb, E);
        float* xo = x_out + 8 * r;
        xo[0] = (float)(v0 * inv_sv); xo[1] = (float)(v1 * inv_sv); xo[2] = (float)(v2 * inv_sv);
        xo[3] = (float)xi[3 * r]; xo[4] = (float)xi[3 * r + 1]; xo[5] = (float)xi[3 * r + 2];
        xo[6] = (float)z[2 * r]; xo[7] = (float)z[2 * r + 1];
        g_out[r] = (float)sqrt(v0 * v0 + v1 * v1 + v2 * v2);
        bool flag;
        const double c = chi_lane<double>(P, q, gl, bb, E, flag);
        if (flag && q.refine) {
            tgt[3 * r] = pending_mark<float>();
            continue;
        }
        if (c != c) count_root_fail(st);
        harvest_target(vr, xi, r, c, tgt, chi_out);
    }
}

struct HarvestJob {
    const double* vr;
    const double* xi;
    const double* z;
    double b_max_A, half_m_over_k;
    float* tgt;
    double* chi_out;
    __device__ int64_t count(int64_t n) const { return n; }
    __device__ bool pending(int64_t r) const { return is_pending(tgt[3 * r]); }
    __device__ void inputs(int64_t r, double& bb, double& E) const
    {
        harvest_b_E(vr, z, b_max_A, half_m_over_k, r, bb, E);
    }
    __device__ void store(int64_t r, double c) const { harvest_target(vr, xi, r, c, tgt, chi_out); }
};

template <class Job>
static int launch_refine(const Job& job, int64_t n, const Pot& P, const QuadCfg& q,
                         const GLRule& gl, dsmc_status* st, hipStream_t s, const char* what)
{
    if (!q.refine || n <= 0) return DSMC_OK;
    int64_t blocks = (n + 255) / 256;
    const int pb = persistent_blocks(256);
    if (blocks > pb) blocks = pb;
    k_refine<Job><<<(int)blocks, 256, 0, s>>>(job, n, P, q, gl, st);
    DSMC_LAUNCH_CHECK(what);
    return DSMC_OK;
}

}  // namespace dsmc

using namespace dsmc;

extern "C" int dsmc_deflect_jager(int64_t n, int32_t dtype, const void* b, const void* g,
                                  void* chi, double m_red, const dsmc_potential* pot,
                                  dsmc_quad quad, int32_t fold, dsmc_status* st,
                                  dsmc_stream_t stream)
{
    if (n < 0) return arg_error("dsmc_deflect_jager: n < 0");
    if (n > 0 && (!b || !g || !chi)) return arg_error("dsmc_deflect_jager: null pointer");
    if (!(m_red > 0)) return arg_error("dsmc_deflect_jager: m_red must be > 0");
    Pot P;
    int rc = get_pot(pot, &P);
    if (rc) return rc;
    QuadCfg q;
    GLRule gl;
    rc = make_cfg(quad, &q, &gl);
    if (rc) return rc;
    if (n == 0) return DSMC_OK;
    const double hmk = 0.5 * m_red / KB;
    hipStream_t s = as_stream(stream);
    int blocks = (int)((n + 255) / 256);
    const int pb = persistent_blocks(256);
    if (blocks > pb) blocks = pb;
    if (dtype == DSMC_F64) {
        k_deflect_f64<<<blocks, 256, 0, s>>>(n, (const double*)b, (const double*)g,
                                                 (double*)chi, hmk, P, q, gl, fold, st);
    } else if (dtype == DSMC_F32) {
        k_deflect_f32<<<blocks, 256, 0, s>>>(n, (const float*)b, (const float*)g, (float*)chi,
                                                hmk, P, q, gl, fold, st);
    } else {
        return arg_error("dsmc_deflect_jager: dtype %d", dtype);
    }
    DSMC_LAUNCH_CHECK("deflect_jager");
    if (dtype == DSMC_F64)
        return launch_refine(DeflectJob<double>{(const double*)b, (const double*)g, (double*)chi,
                                                hmk, fold},
                             n, P, q, gl, st, s, "deflect_jager:refine");
    return launch_refine(DeflectJob<float>{(const float*)b, (const float*)g, (float*)chi, hmk, fold},
                         n, P, q, gl, st, s, "deflect_jager:refine");
}

extern "C" int dsmc_collide_jager(int32_t n_cells, int32_t dtype, dsmc_vec3 v, dsmc_pairs pairs,
                                  dsmc_rng rng, double m_red, double b_max,
                                  const dsmc_potential* pot, dsmc_quad quad, int32_t schedule,
                                  void* ws, size_t ws_bytes, dsmc_status* st,
                                  dsmc_stream_t stream)
{
    int rc = check_pairs("dsmc_collide_jager", n_cells, v, pairs, dtype, ws, ws_bytes);
    if (rc) return rc;
    if (!(m_red > 0) || !(b_max > 0)) return arg_error("dsmc_collide_jager: m_red, b_max > 0");
    if (schedule < DSMC_SCHED_AUTO || schedule > DSMC_SCHED_WAVE)
        return arg_error("dsmc_collide_jager: schedule %d", schedule);
    Pot P;
    rc = get_pot(pot, &P);
    if (rc) return rc;
    QuadCfg q;
    GLRule gl;
    rc = make_cfg(quad, &q, &gl);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    const PairsView pr = PairsView::of(pairs);
    const int pb = persistent_blocks(256);
    const double hmk = 0.5 * m_red / KB;
    if (dtype == DSMC_F64) {
        k_phaseA_jager_f64<<<pb, 256, 0, s>>>(n_cells, pr, rng, v3<const double>(v), hmk,
                                                 b_max * 1e10, P, q, gl,
                                                 PairBuf<double>::of(ws, pairs.cap), st);
    } else {
        k_phaseA_jager_f32<<<pb, 256, 0, s>>>(n_cells, pr, rng, v3<const float>(v), hmk,
                                                b_max * 1e10, P, q, gl,
                                                PairBuf<float>::of(ws, pairs.cap), st);
    }
    DSMC_LAUNCH_CHECK("collide_jager:phaseA");
    if (dtype == DSMC_F64)
        rc = launch_refine(PhaseAJagerJob<double>{pr, rng, v3<const double>(v), hmk, b_max * 1e10,
                                                  PairBuf<double>::of(ws, pairs.cap), n_cells},
                           pairs.cap, P, q, gl, st, s, "collide_jager:refine");
    else
        rc = launch_refine(PhaseAJagerJob<float>{pr, rng, v3<const float>(v), hmk, b_max * 1e10,
                                                 PairBuf<float>::of(ws, pairs.cap), n_cells},
                           pairs.cap, P, q, gl, st, s, "collide_jager:refine");
    if (rc) return rc;
    if (schedule == DSMC_SCHED_DEFER) return DSMC_OK;
    return phase_b(RULE_CHI, dtype, n_cells, nullptr, v, pairs, ws, pairs.cap, schedule, s);
}

extern "C" int dsmc_harvest_rows(int64_t B, const double* vr, const double* xi, const double* z,
                                 double sigma_v, double b_max, double m_red,
                                 const dsmc_potential* pot, dsmc_quad quad, float* x_out,
                                 float* g_out, float* target_out, double* chi_out,
                                 dsmc_status* st, dsmc_stream_t stream)
{
    if (B < 0) return arg_error("dsmc_harvest_rows: B < 0");
    if (B > 0 && (!vr || !xi || !z || !x_out || !g_out || !target_out))
        return arg_error("dsmc_harvest_rows: null pointer");
    if (!(sigma_v > 0) || !(b_max > 0) || !(m_red > 0))
        return arg_error("dsmc_harvest_rows: sigma_v, b_max, m_red must be > 0");
    Pot P;
    int rc = get_pot(pot, &P);
    if (rc) return rc;
    QuadCfg q;
    GLRule gl;
    rc = make_cfg(quad, &q, &gl);
    if (rc) return rc;
    if (B == 0) return DSMC_OK;
    int blocks = (int)((B + 255) / 256);
    const int pb = persistent_blocks(256);
    if (blocks > pb) blocks = pb;
    k_harvest<<<blocks, 256, 0, as_stream(stream)>>>(B, vr, xi, z, 1.0 / sigma_v, b_max * 1e10,
                                                     0.5 * m_red / KB, P, q, gl, x_out, g_out,
                                                     target_out, chi_out, st);
    DSMC_LAUNCH_CHECK("harvest_rows");
    return launch_refine(HarvestJob{vr, xi, z, b_max * 1e10, 0.5 * m_red / KB, target_out, chi_out},
                         B, P, q, gl, st, as_stream(stream), "harvest_rows:refine");
}

// ------------------------------------------------------------------------
// Chapman-Enskog viscosity (section "Macroscopic Validation: Viscosity and
// Transport Coefficients"): transport cross-section
//   Q2(E) = 2 pi int_0^b_cut (1 - cos^2 chi) b db
// by composite Gauss-Legendre in b (chi from the quadrature above, FP64, the
// wave-cooperative refinement included), the Maxwellian average by
// generalised Gauss-Laguerre in x = E / kT, and mu = 5/16 sqrt(pi m k T) / Omega.
// ------------------------------------------------------------------------
namespace dsmc {

constexpr int LAG_MAX = 64;

struct LagRule {
    int n;
    double x[LAG_MAX];
    double w[LAG_MAX];
};

// Generalised Gauss-Laguerre nodes and weights (weight x^alpha e^-x): nodes
// are the eigenvalues of the symmetric tridiagonal Jacobi matrix (diagonal
// 2k + alpha + 1, off-diagonal sqrt(k (k + alpha))), found by cyclic Jacobi
// rotations (Golub-Welsch); weights from the closed form in L_{n+1}.
static int make_laguerre(int n, double alpha, LagRule* L)
{
    if (n < 1 || n > LAG_MAX) return arg_error("laguerre: n %d not in [1, %d]", n, LAG_MAX);
    std::vector<double> A((size_t)n * n, 0.0);
    for (int k = 0; k < n; ++k) {
        A[(size_t)k * n + k] = 2.0 * k + alpha + 1.0;
        if (k > 0) {
            const double b = sqrt(k * (k + alpha));
            A[(size_t)k * n + k - 1] = b;
            A[(size_t)(k - 1) * n + k] = b;
        }
    }
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += A[(size_t)p * n + q] * A[(size_t)p * n + q];
        if (off < 1e-30) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (fabs(apq) < 1e-300) continue;
                const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                const double theta = 0.5 * (aqq - app) / apq;
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {  // columns p, q
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - s * akq;
                    A[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // rows p, q
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - s * aqk;
                    A[(size_t)q * n + k] = s * apk + c * aqk;
                }
            }
    }
    // weights from the closed form Gamma(n+alpha+1) x / (n! (n+1)^2 L_{n+1}(x)^2)
    // (more accurate on the tiny weights than squared eigenvector components)
    L->n = n;
    const double lg = lgamma(n + alpha + 1.0) - lgamma(n + 1.0) - 2.0 * log(n + 1.0);
    for (int k = 0; k < n; ++k) {
        const double x = A[(size_t)k * n + k];
        double p0 = 1.0, p1 = 1.0 + alpha - x;
        for (int j = 2; j <= n + 1; ++j) {
            const double p2 = ((2.0 * j - 1.0 + alpha - x) * p1 - (j - 1.0 + alpha) * p0) / j;
            p0 = p1;
            p1 = p2;
        }
        L->x[k] = x;
        L->w[k] = exp(lg) * x / (p1 * p1);
    }
    return DSMC_OK;
}

// One term of the b integral: node j of energy i (b in Angstrom).
__global__ void __launch_bounds__(256)
k_q2_terms(int64_t n_items, int n_b, const double* __restrict__ E_kelvin, double b_cut_A,
           int n_panels, GLRule bgl, Pot P, QuadCfg q, GLRule gl, double* __restrict__ terms,
           dsmc_status* st)
{
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~63); base < n_items;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t it = base + (threadIdx.x & 63);
        const bool active = it < n_items;
        const int64_t i = active ? it / n_b : 0;
        const int j = active ? (int)(it % n_b) : 0;
        const int pnl = j / bgl.n, node = j % bgl.n;
        const double h = b_cut_A / n_panels;
        const double b = h * (pnl + bgl.t[node]);
        const double E = active ? E_kelvin[i] : 1.0;
        double c = chi_wave_inplace(P, q, gl, b, E, active);
        if (!active) continue;
        if (c != c) {
            if (st) {
                atomicAdd(&st->root_fail, 1);
                atomicOr(&st->flags, (uint32_t)DSMC_ST_ROOT_FAIL);
            }
            c = 0.0;
        }
        const double cc = cos(c);
        terms[it] = h * bgl.w[node] * (1.0 - cc * cc) * b;
    }
}

// Q2[i] = 2 pi sum_j terms[i][j] (fixed order), in m^2.
__global__ void __launch_bounds__(256)
k_q2_sum(int64_t n_E, int n_b, const double* __restrict__ terms, double* __restrict__ Q)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_E;
         i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < n_b; ++j) s += terms[i * n_b + j];
        Q[i] = 2.0 * 3.14159265358979323846 * s * 1e-20;
    }
}

__global__ void __launch_bounds__(256)
k_ce_energies(int n_T, const double* __restrict__ T, LagRule lag, double* __restrict__ E)
{
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n_T * lag.n;
         q += gridDim.x * blockDim.x)
        E[q] = lag.x[q % lag.n] * T[q / lag.n];
}

__global__ void __launch_bounds__(256)
k_ce_finish(int n_T, const double* __restrict__ T, LagRule lag, double scale, double m,
            const double* __restrict__ Q, double* __restrict__ omega, double* __restrict__ mu)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_T; i += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < lag.n; ++k) s += lag.w[k] * Q[(int64_t)i * lag.n + k];
        const double om = scale * s;
        omega[i] = om;
        mu[i] = 5.0 / 16.0 * sqrt(3.14159265358979323846 * m * KB * T[i]) / om;
    }
}

static int q2_impl(int64_t n_E, const double* E, double b_cut, int n_panels, int n_gl,
                   const dsmc_potential* pot, const dsmc_quad& quad, double* Q, void* ws,
                   dsmc_status* st, hipStream_t s)
{
    Pot P;
    int rc = get_pot(pot, &P);
    if (rc) return rc;
    QuadCfg q;
    GLRule gl, bgl;
    rc = make_cfg(quad, &q, &gl);
    if (rc) return rc;
    rc = make_gl(n_gl, &bgl);
    if (rc) return rc;
    const int n_b = n_panels * n_gl;
    const int64_t items = n_E * (int64_t)n_b;
    double* terms = static_cast<double*>(ws);
    const int pb = persistent_blocks(256);
    int64_t blocks = (items + 255) / 256;
    if (blocks > pb) blocks = pb;
    k_q2_terms<<<(int)(blocks < 1 ? 1 : blocks), 256, 0, s>>>(items, n_b, E, b_cut * 1e10,
                                                              n_panels, bgl, P, q, gl, terms, st);
    DSMC_LAUNCH_CHECK("q2:terms");
    k_q2_sum<<<(int)((n_E + 255) / 256), 256, 0, s>>>(n_E, n_b, terms, Q);
    DSMC_LAUNCH_CHECK("q2:sum");
    return DSMC_OK;
}

static int check_q2_args(const char* who, double b_cut, int n_panels, int n_gl)
{
    if (!(b_cut > 0)) return arg_error("%s: b_cut must be > 0", who);
    if (n_panels < 1 || n_panels > (1 << 20)) return arg_error("%s: n_panels %d", who, n_panels);
    if (n_gl < 2 || n_gl > GL_MAX) return arg_error("%s: n_gl %d", who, n_gl);
    return DSMC_OK;
}

}  // namespace dsmc

extern "C" size_t dsmc_transport_q2_ws(int64_t n_E, int32_t n_panels, int32_t n_gl)
{
    if (n_E < 0 || n_panels < 1 || n_gl < 1) return 0;
    return align_up(sizeof(double) * (size_t)n_E * n_panels * n_gl) + 256;
}

extern "C" int dsmc_transport_q2(int64_t n_E, const double* E_kelvin, double b_cut,
                                 int32_t n_panels, int32_t n_gl, const dsmc_potential* pot,
                                 dsmc_quad quad, double* Q, void* ws, size_t ws_bytes,
                                 dsmc_status* st, dsmc_stream_t stream)
{
    int rc = check_q2_args("dsmc_transport_q2", b_cut, n_panels, n_gl);
    if (rc) return rc;
    if (n_E < 0) return arg_error("dsmc_transport_q2: n_E < 0");
    if (n_E == 0) return DSMC_OK;
    if (!E_kelvin || !Q || !ws) return arg_error("dsmc_transport_q2: null pointer");
    if (ws_bytes < dsmc_transport_q2_ws(n_E, n_panels, n_gl))
        return arg_error("dsmc_transport_q2: workspace too small");
    return q2_impl(n_E, E_kelvin, b_cut, n_panels, n_gl, pot, quad, Q, ws, st, as_stream(stream));
}

extern "C" size_t dsmc_viscosity_ce_ws(int32_t n_T, int32_t n_panels, int32_t n_gl, int32_t n_lag)
{
    if (n_T < 0 || n_lag < 1) return 0;
    const int64_t nE = (int64_t)n_T * n_lag;
    return 2 * align_up(sizeof(double) * (size_t)nE) + dsmc_transport_q2_ws(nE, n_panels, n_gl);
}

extern "C" int dsmc_viscosity_ce(int32_t n_T, const double* T, double m, double b_cut,
                                 int32_t n_panels, int32_t n_gl, int32_t n_lag, int32_t mode,
                                 const dsmc_potential* pot, dsmc_quad quad, double* omega,
                                 double* mu, void* ws, size_t ws_bytes, dsmc_status* st,
                                 dsmc_stream_t stream)
{
    int rc = check_q2_args("dsmc_viscosity_ce", b_cut, n_panels, n_gl);
    if (rc) return rc;
    if (n_T < 0 || !(m > 0)) return arg_error("dsmc_viscosity_ce: n_T >= 0 and m > 0 required");
    if (mode != DSMC_CE_STANDARD && mode != DSMC_CE_AS_PRINTED)
        return arg_error("dsmc_viscosity_ce: mode %d", mode);
    if (n_T == 0) return DSMC_OK;
    if (!T || !omega || !mu || !ws) return arg_error("dsmc_viscosity_ce: null pointer");
    if (ws_bytes < dsmc_viscosity_ce_ws(n_T, n_panels, n_gl, n_lag))
        return arg_error("dsmc_viscosity_ce: workspace too small");
    LagRule lag;
    const bool printed = mode == DSMC_CE_AS_PRINTED;
    rc = make_laguerre(n_lag, printed ? 2.0 : 3.0, &lag);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    const int64_t nE = (int64_t)n_T * n_lag;
    uint8_t* w = static_cast<uint8_t*>(ws);
    double* E = reinterpret_cast<double*>(w);
    w += align_up(sizeof(double) * (size_t)nE);
    double* Q = reinterpret_cast<double*>(w);
    w += align_up(sizeof(double) * (size_t)nE);
    k_ce_energies<<<(int)((nE + 255) / 256), 256, 0, s>>>(n_T, T, lag, E);
    DSMC_LAUNCH_CHECK("ce:energies");
    rc = q2_impl(nE, E, b_cut, n_panels, n_gl, pot, quad, Q, w, st, s);
    if (rc) return rc;
    k_ce_finish<<<(n_T + 255) / 256, 256, 0, s>>>(n_T, T, lag, printed ? 0.5 : 0.25, m, Q, omega,
                                                  mu);
    DSMC_LAUNCH_CHECK("ce:finish");
    return DSMC_OK;
}
