// Ab initio deflection angle by quadrature of the classical deflection
// integral (section "Computational Implementation: The Exact vs. Neural
// Paradigm"), one lane per pair, no cross-lane traffic:
//   1. E = m_red g^2 / 2; r_min = largest root of D(r) = 1 - b^2/r^2 - V(r)/E,
//      bracketed by a downward geometric scan (fine steps at low energy, where
//      D can have several roots) and refined by safeguarded Newton steps.
//   2. u = r_min / r maps the range to [0, 1]; u = 1 - t^2 removes the
//      inverse-square-root singularity at u = 1, leaving the smooth integrand
//      2 t / sqrt(F) with F = beta^2 t^2 (2 - t^2) + (V(r_min) - V(r))/E,
//      beta = b / r_min, which is integrated by fixed-order Gauss-Legendre.
//   3. chi = pi - 2 beta * integral.
// Near r_min the potential difference is formed as -int V' dr (2-point
// Gauss-Legendre) to avoid cancellation.
#include <math.h>

#include <string.h>

#include <vector>

#include "collide.hpp"

namespace dsmc {

constexpr int GL_MAX = 128;

struct GLRule {
    int n;
    double t[GL_MAX];
    double w[GL_MAX];
};

// Potential and the derived quantities a kernel needs.
struct Pot {
    dsmc_potential p;
    double r_sw;     // short-range switch 0.4 R_eps (JAGER)
    double r_zero;   // largest zero of V (JAGER); V < 0 beyond it
    double e_scan;   // below this E (K), D may have several roots: fine scan
    double fact[17]; // 1/k!
};

struct QuadCfg {
    int max_iter;
    int low_panels;
    double scan_ratio;
};

// ------------------------------------------------------------------------
// Potential (T arithmetic)
// ------------------------------------------------------------------------
// Beyond beta_tt r = 60 every Tang-Toennies factor f_6..f_16 is 1 to better
// than 1e-13 (the tail exp(-x) sum x^k/k! is below that), so they are taken
// as 1 there.
constexpr double DAMP_OFF = 60.0;
template <typename T>
__device__ __forceinline__ T dexp(T x) { return exp(x); }
template <>
__device__ __forceinline__ float dexp<float>(float x) { return expf(x); }

template <typename T>
__device__ __forceinline__ T V_of(const Pot& P, T r)
{
    const dsmc_potential& p = P.p;
    if (p.kind == DSMC_POT_INVPOW) {
        T rn = r;
        for (int q = 1; q < p.n; ++q) rn *= r;
        return T(p.K) / rn;
    }
    if (r < T(P.r_sw)) return T(p.A_sr) / r * dexp<T>(-T(p.a_sr) * r);
    const T ri = T(1) / r;
    const T rep = T(p.A) * dexp<T>(T(p.a1) * r + T(p.a2) * r * r + T(p.am1) * ri + T(p.am2) * ri * ri);
    const T x = T(p.beta_tt) * r;
    const T ri2 = ri * ri;
    T rpow = ri2 * ri2 * ri2;  // r^-6
    T disp = T(0);
    if (x >= T(DAMP_OFF)) {
        // damping factors equal 1 to well below rounding (and x^16 would
        // overflow FP32 at large r)
#pragma unroll
        for (int n = 0; n < 6; ++n) {
            disp += T(p.C[n]) * rpow;
            rpow *= ri2;
        }
        return rep - disp;
    }
    const T ex = dexp<T>(-x);
    T term = T(1), S = T(1);
#pragma unroll
    for (int k = 1; k <= 16; ++k) {
        term = term * x * T(1.0 / k);  // x^k / k!
        S += term;
        if (k >= 6 && (k & 1) == 0) {
            disp += (T(1) - ex * S) * T(p.C[(k - 6) / 2]) * rpow;
            rpow *= ri2;
        }
    }
    return rep - disp;
}

template <typename T>
__device__ __forceinline__ T dV_of(const Pot& P, T r)
{
    const dsmc_potential& p = P.p;
    if (p.kind == DSMC_POT_INVPOW) {
        T rn = r;
        for (int q = 1; q < p.n; ++q) rn *= r;
        return -T(p.n) * T(p.K) / (rn * r);
    }
    const T ri = T(1) / r;
    if (r < T(P.r_sw)) {
        const T v = T(p.A_sr) * ri * dexp<T>(-T(p.a_sr) * r);
        return -v * (T(p.a_sr) + ri);
    }
    const T phi_r = T(p.a1) + T(2) * T(p.a2) * r - T(p.am1) * ri * ri - T(2) * T(p.am2) * ri * ri * ri;
    const T rep = T(p.A) * dexp<T>(T(p.a1) * r + T(p.a2) * r * r + T(p.am1) * ri + T(p.am2) * ri * ri);
    const T x = T(p.beta_tt) * r;
    const T ri2 = ri * ri;
    T rpow = ri2 * ri2 * ri2;
    T dd = T(0);
    if (x >= T(DAMP_OFF)) {
#pragma unroll
        for (int n = 0; n < 6; ++n) {
            dd -= T(6 + 2 * n) * T(p.C[n]) * rpow * ri;
            rpow *= ri2;
        }
        return rep * phi_r - dd;
    }
    const T ex = dexp<T>(-x);
    T term = T(1), S = T(1);
#pragma unroll
    for (int k = 1; k <= 16; ++k) {
        term = term * x * T(1.0 / k);  // x^k / k!
        S += term;
        if (k >= 6 && (k & 1) == 0) {
            // d/dr [f_k(beta r) C_k r^-k], f_k'(x) = e^-x x^k / k!
            dd += T(p.C[(k - 6) / 2]) * (T(p.beta_tt) * ex * term * rpow -
                                        T(k) * (T(1) - ex * S) * rpow * ri);
            rpow *= ri2;
        }
    }
    return rep * phi_r - dd;
}

template <typename T> struct Consts;
template <> struct Consts<double> {
    static constexpr double pi = 3.14159265358979323846;
    static constexpr double rtol = 4e-16;
};
template <> struct Consts<float> {
    static constexpr float pi = 3.14159265358979f;
    static constexpr float rtol = 2e-7f;
};

// D(r) = 1 - b^2/r^2 - V(r)/E
template <typename T>
__device__ __forceinline__ T D_of(const Pot& P, T b2, T E, T r)
{
    return T(1) - b2 / (r * r) - V_of<T>(P, r) / E;
}

// One node of the t integral: 2 t / sqrt(F) with
// F = beta^2 t^2 (2 - t^2) + (V(r_min) - V(r))/E + D0 and r = r_min / (1 - t^2);
// also F / t^2 (for the peak indicator).
template <typename T>
__device__ __forceinline__ T node_term(const Pot& P, T rmin, T beta, T Vmin, T E, T D0, T t,
                                       T& f_over_t2)
{
    const T g1 = T(0.5) - T(0.28867513459481287);  // 2-point Gauss-Legendre on [0,1]
    const T g2 = T(0.5) + T(0.28867513459481287);
    const T t2 = t * t;
    const T dr = rmin * t2 / (T(1) - t2);
    T dV = T(0);
    if (P.p.kind != DSMC_POT_HS) {
        if (t2 < T(1e-3))
            dV = -dr * T(0.5) * (dV_of<T>(P, rmin + g1 * dr) + dV_of<T>(P, rmin + g2 * dr));
        else
            dV = Vmin - V_of<T>(P, rmin + dr);
    }
    const T F = beta * beta * t2 * (T(2) - t2) + dV / E + D0;
    f_over_t2 = F / t2;
    return F > T(0) ? T(2) * t / sqrt(F) : T(0);
}

// Gauss-Legendre over t in [ta, tb]; qmin tracks min F / t^2 over the nodes.
template <typename T>
__device__ __forceinline__ T integral_part(const Pot& P, const GLRule& gl, T rmin, T beta, T Vmin,
                                           T E, T D0, T ta, T tb, T& qmin)
{
    const T len = tb - ta;
    T I = T(0);
    for (int k = 0; k < gl.n; ++k) {
        T fq;
        I += T(gl.w[k]) * node_term<T>(P, rmin, beta, Vmin, E, D0, ta + len * T(gl.t[k]), fq);
        qmin = fq < qmin ? fq : qmin;
    }
    return len * I;
}

// Peak indicator threshold: below the scan energy, F / t^2 (which is
// r_min D'(r_min) at t = 0 and 1 at t = 1) dipping under this value marks an
// integrand with a sharp interior peak (near orbiting), for which one
// Gauss-Legendre panel is not enough; such pairs are re-integrated on
// low_panels equal panels.
constexpr double Q_REFINE = 0.6;

template <typename T>
struct QuadState {
    T rmin, beta, Vmin, E, D0;
    bool refine;
};

// chi(b, E) with b in Angstrom, E/k_B in K, by the one-panel rule; returns
// NaN if no root is found.  s receives what a panel refinement needs.
template <typename T>
__device__ T chi_quad_std(const Pot& P, const QuadCfg& q, const GLRule& gl, T b, T E,
                          QuadState<T>& s)
{
    const T pi = Consts<T>::pi;
    const T b2 = b * b;
    s.refine = false;
    T rmin, D0 = T(0);
    if (P.p.kind == DSMC_POT_HS) {
        const T d = T(P.p.d);
        rmin = b > d ? b : d;
        const T beta = b / rmin;
        D0 = b > d ? T(0) : T(1) - beta * beta;
    } else {
        T rhi;
        if (P.p.kind == DSMC_POT_JAGER) {
            rhi = b > T(P.r_zero) ? b : T(P.r_zero);
        } else {
            const T rk = pow(T(2) * T(P.p.K) / E, T(1) / T(P.p.n));
            rhi = T(2) * b > rk ? T(2) * b : rk;
            if (!(rhi > T(0))) rhi = T(1);
        }
        T fhi = D_of<T>(P, b2, E, rhi);
        if (fhi <= T(0)) {
            rmin = rhi;
        } else {
            const T ratio = (E < T(P.e_scan)) ? T(q.scan_ratio) : T(0.7);
            T rlo = rhi, flo = fhi;
            bool found = false;
            for (int it = 0; it < 4000; ++it) {
                rlo = rhi * ratio;
                flo = D_of<T>(P, b2, E, rlo);
                if (flo <= T(0)) { found = true; break; }
                rhi = rlo;
                fhi = flo;
                if (rlo < T(1e-4)) break;
            }
            if (!found) return T(NAN);
            // safeguarded Newton inside [rlo, rhi], D(rlo) <= 0 < D(rhi)
            T r = rhi;
            for (int it = 0; it < q.max_iter; ++it) {
                const T f = D_of<T>(P, b2, E, r);
                if (f > T(0)) rhi = r; else rlo = r;
                const T fp = T(2) * b2 / (r * r * r) - dV_of<T>(P, r) / E;
                T rn = r - f / fp;
                if (!(rn > rlo && rn < rhi)) rn = T(0.5) * (rlo + rhi);
                const T step = rn - r;
                r = rn;
                if (fabs(step) <= Consts<T>::rtol * r || rhi - rlo <= Consts<T>::rtol * r) break;
            }
            rmin = r;
        }
    }
    const T beta = b / rmin;
    const T Vmin = (P.p.kind == DSMC_POT_HS) ? T(0) : V_of<T>(P, rmin);
    s.rmin = rmin;
    s.beta = beta;
    s.Vmin = Vmin;
    s.E = E;
    s.D0 = D0;
    T I = T(0);
    T qmin = T(1e30);
    if (E < T(P.e_scan) && P.p.kind == DSMC_POT_JAGER) {
        // low energy: r_min lies outside the short-range region
        I = integral_part<T>(P, gl, rmin, beta, Vmin, E, D0, T(0), T(1), qmin);
        s.refine = q.low_panels > 1 && qmin < T(Q_REFINE);
    } else {
        // the short-range switch of the JAGER form is a kink of the
        // integrand: integrate the two sides separately
        T tsw = T(1);
        if (P.p.kind == DSMC_POT_JAGER && rmin < T(P.r_sw)) tsw = sqrt(T(1) - rmin / T(P.r_sw));
        I = integral_part<T>(P, gl, rmin, beta, Vmin, E, D0, T(0), tsw, qmin);
        if (tsw < T(1)) I += integral_part<T>(P, gl, rmin, beta, Vmin, E, D0, tsw, T(1), qmin);
    }
    return pi - T(2) * beta * I;
}

// chi for the lanes of a wave (all 64 lanes call it; inactive lanes pass
// active = false).  Pairs flagged for refinement are re-integrated one at a
// time by the whole wave: the low_panels x n nodes are spread over the lanes
// and summed by a fixed butterfly, so the cost of a flagged pair is a few
// node evaluations per lane.
template <typename T>
__device__ T chi_quad_wave(const Pot& P, const QuadCfg& q, const GLRule& gl, T b, T E,
                           bool active)
{
    QuadState<T> s{};
    T c = T(0);
    if (active) c = chi_quad_std<T>(P, q, gl, b, E, s);
    const bool flag = active && s.refine && c == c;
    uint64_t pend = __ballot(flag);
    const int lane = threadIdx.x & 63;
    const int n = gl.n, np = q.low_panels, total = n * np;
    const T inv_np = T(1) / T(np);
    while (pend) {
        const int src = __ffsll((unsigned long long)pend) - 1;
        const T rmin = __shfl(s.rmin, src, 64), beta = __shfl(s.beta, src, 64);
        const T Vmin = __shfl(s.Vmin, src, 64), Ee = __shfl(s.E, src, 64);
        const T D0 = __shfl(s.D0, src, 64);
        T I = T(0);
        for (int m = lane; m < total; m += 64) {
            const int k = m / n, j = m - k * n;
            T fq;
            I += T(gl.w[j]) * inv_np *
                 node_term<T>(P, rmin, beta, Vmin, Ee, D0, (T(k) + T(gl.t[j])) * inv_np, fq);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) I += __shfl_xor(I, o, 64);
        if (lane == src) c = Consts<T>::pi - T(2) * beta * I;
        pend &= pend - 1;
    }
    return c;
}

// ------------------------------------------------------------------------
// Host side: Gauss-Legendre nodes by Newton on P_n, potential set-up.
// ------------------------------------------------------------------------
static int make_gl(int n, GLRule* g)
{
    if (n == 0) n = 64;
    if (n < 2 || n > GL_MAX) return arg_error("dsmc_quad: n_nodes %d not in [2, %d]", n, GL_MAX);
    g->n = n;
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double x = cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                const double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        // recompute derivative at the converged node
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; ++k) {
            const double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = pk;
        }
        dp = n * (x * p1 - p0) / (x * x - 1.0);
        // map [-1, 1] -> [0, 1]
        g->t[i] = 0.5 * (1.0 - x);
        g->w[i] = 1.0 / ((1.0 - x * x) * dp * dp);  // (2 / ((1-x^2) P'^2)) / 2
    }
    return DSMC_OK;
}

static double host_V(const Pot& P, double r)
{
    const dsmc_potential& p = P.p;
    if (r < P.r_sw) return p.A_sr / r * exp(-p.a_sr * r);
    double rep = p.A * exp(p.a1 * r + p.a2 * r * r + p.am1 / r + p.am2 / (r * r));
    double x = p.beta_tt * r, ex = exp(-x), term = 1, S = 1, disp = 0;
    for (int k = 1; k <= 16; ++k) {
        term *= x / k;
        S += term;
        if (k >= 6 && k % 2 == 0) disp += (1 - ex * S) * p.C[(k - 6) / 2] / pow(r, k);
    }
    return rep - disp;
}

static int make_pot(const dsmc_potential* pot, Pot* P)
{
    if (!pot) return arg_error("dsmc potential: null");
    P->p = *pot;
    P->fact[0] = 1.0;
    for (int k = 1; k <= 16; ++k) P->fact[k] = P->fact[k - 1] * k;
    P->r_sw = 0.0;
    P->r_zero = 0.0;
    P->e_scan = 0.0;
    switch (pot->kind) {
    case DSMC_POT_HS:
        if (!(pot->d > 0)) return arg_error("dsmc potential: HS diameter must be > 0");
        return DSMC_OK;
    case DSMC_POT_INVPOW:
        if (pot->n < 1 || pot->n > 12 || !(pot->K >= 0))
            return arg_error("dsmc potential: INVPOW needs 1 <= n <= 12 and K >= 0");
        return DSMC_OK;
    case DSMC_POT_JAGER: {
        if (!(pot->R_eps > 0) || !(pot->A > 0) || !(pot->beta_tt > 0))
            return arg_error("dsmc potential: bad JAGER parameters");
        P->r_sw = 0.4 * pot->R_eps;
        // largest zero of V: scan in from 50 A, then bisect
        double hi = 50.0, lo = 50.0;
        while (host_V(*P, lo) <= 0.0 && lo > 0.05) lo *= 0.99;
        if (host_V(*P, lo) <= 0.0) return arg_error("dsmc potential: V has no repulsive core");
        for (int it = 0; it < 200; ++it) {
            const double m = 0.5 * (lo + hi);
            if (host_V(*P, m) > 0.0) lo = m; else hi = m;
        }
        P->r_zero = hi;
        // Energy above which r^2 (1 - V(r)/E) is increasing in r on the
        // outer region (single turning point for every b); below it the root
        // scan must be fine.  Found on a grid, then doubled for margin.
        double ecrit = 0.0;
        for (double E = 1.0; E < 1e5; E *= 1.05) {
            bool mono = true;
            double prev = -1e300;
            for (double r = 0.6 * P->r_zero; r < 40.0; r *= 1.002) {
                const double B = r * r * (1.0 - host_V(*P, r) / E);
                if (B < prev) { mono = false; break; }
                prev = B;
            }
            if (mono) { ecrit = E; break; }
        }
        P->e_scan = ecrit > 0 ? 2.0 * ecrit : 1e30;
        return DSMC_OK;
    }
    }
    return arg_error("dsmc potential: kind %d", pot->kind);
}

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

static int make_cfg(const dsmc_quad& q, QuadCfg* c, GLRule* gl)
{
    c->max_iter = q.max_iter > 0 ? q.max_iter : 60;
    c->scan_ratio = q.scan_ratio > 0 ? q.scan_ratio : 0.98;
    c->low_panels = q.low_panels > 0 ? q.low_panels : 4;
    if (c->low_panels > 16) return arg_error("dsmc_quad: low_panels %d > 16", c->low_panels);
    if (!(c->scan_ratio > 0.5 && c->scan_ratio < 1.0))
        return arg_error("dsmc_quad: scan_ratio %g not in (0.5, 1)", c->scan_ratio);
    return make_gl(q.n_nodes, gl);
}

constexpr double KB = 1.380649e-23;

// ------------------------------------------------------------------------
// Kernels
// ------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_deflect(int64_t n, const T* __restrict__ b, const T* __restrict__ g, T* __restrict__ chi,
          T half_m_over_k, Pot P, QuadCfg q, GLRule gl, int fold, dsmc_status* st)
{
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~63); base < n;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = base + (threadIdx.x & 63);
        const bool active = p < n;
        const T gg = active ? g[p] : T(1);
        const T E = half_m_over_k * gg * gg;
        T c = chi_quad_wave<T>(P, q, gl, active ? b[p] * T(1e10) : T(1), E, active);
        if (!active) continue;
        if (c != c) {
            if (st) {
                atomicAdd(&st->root_fail, 1);
                atomicOr(&st->flags, (uint32_t)DSMC_ST_ROOT_FAIL);
            }
        } else if (fold) {
            c = acos(cos(c));
        }
        chi[p] = c;
    }
}

// Phase A of the in-step ab initio rule.
template <typename T>
__global__ void __launch_bounds__(256)
k_phaseA_jager(int32_t n_cells, PairsView pr, dsmc_rng rng, V3<const T> v, T half_m_over_k,
               T b_max_A, Pot P, QuadCfg q, GLRule gl, PairBuf<T> out, dsmc_status* st)
{
    const int64_t np = pr.total(n_cells);
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~63); base < np;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = base + (threadIdx.x & 63);
        const bool active = p < np;
        T xi[3] = {T(0), T(0), T(0)}, z[2], u4 = T(0);
        T E = T(1), bb = T(1);
        if (active) {
            const int32_t k = pr.cell[p];
            const uint32_t a = (uint32_t)(p - pr.off[k]);
            pair_latents(rng, a, (uint32_t)k, xi, z, u4);
            const int32_t i = pr.i[p], j = pr.j[p];
            const T rx = v.x[i] - v.x[j], ry = v.y[i] - v.y[j], rz = v.z[i] - v.z[j];
            const T g2 = rx * rx + ry * ry + rz * rz;
            E = half_m_over_k * g2;
            bb = b_max_A * sqrt(u4);  // b^2 / b_max^2 = 1 - exp(-|z|^2/2) = U4
        }
        T c = chi_quad_wave<T>(P, q, gl, bb, E, active);
        if (!active) continue;
        if (c != c) {
            if (st) {
                atomicAdd(&st->root_fail, 1);
                atomicOr(&st->flags, (uint32_t)DSMC_ST_ROOT_FAIL);
            }
            c = T(0);  // no deflection for a failed evaluation
        }
        out.a[p] = cos(c);
        out.b[p] = sin(c);
        out.c[p] = xi[0];
        out.d[p] = xi[1];
        out.e[p] = xi[2];
    }
}

// Harvest rows: targets from the quadrature.
__global__ void __launch_bounds__(256)
k_harvest(int64_t B, const double* __restrict__ vr, const double* __restrict__ xi,
          const double* __restrict__ z, double inv_sv, double b_max_A, double half_m_over_k,
          Pot P, QuadCfg q, GLRule gl, float* __restrict__ x_out, float* __restrict__ g_out,
          float* __restrict__ tgt, double* __restrict__ chi_out, dsmc_status* st)
{
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~63); base < B;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = base + (threadIdx.x & 63);
        const bool active = r < B;
        const int64_t rr = active ? r : 0;
        const double v0 = vr[3 * rr], v1 = vr[3 * rr + 1], v2 = vr[3 * rr + 2];
        const double x0 = xi[3 * rr], x1 = xi[3 * rr + 1], x2 = xi[3 * rr + 2];
        const double z0 = z[2 * rr], z1 = z[2 * rr + 1];
        double vh[3], e[3];
        const double g = unit3<double>(v0, v1, v2, vh);
        const double bt2 = -expm1(-0.5 * (z0 * z0 + z1 * z1));
        const double bb = b_max_A * sqrt(bt2);
        double c = chi_quad_wave<double>(P, q, gl, bb, half_m_over_k * g * g, active);
        if (!active) continue;
        if (c != c) {
            if (st) {
                atomicAdd(&st->root_fail, 1);
                atomicOr(&st->flags, (uint32_t)DSMC_ST_ROOT_FAIL);
            }
        }
        const double xv[3] = {x0, x1, x2};
        perp_dir<double>(xv, vh, e);
        const double cc = cos(c), sc = sin(c);
        for (int d = 0; d < 3; ++d) tgt[3 * r + d] = (float)(g * (cc * vh[d] + sc * e[d]));
        float* xo = x_out + 8 * r;
        xo[0] = (float)(v0 * inv_sv); xo[1] = (float)(v1 * inv_sv); xo[2] = (float)(v2 * inv_sv);
        xo[3] = (float)x0; xo[4] = (float)x1; xo[5] = (float)x2;
        xo[6] = (float)z0; xo[7] = (float)z1;
        g_out[r] = (float)g;
        if (chi_out) chi_out[r] = c;
    }
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
        k_deflect<double><<<blocks, 256, 0, s>>>(n, (const double*)b, (const double*)g,
                                                 (double*)chi, hmk, P, q, gl, fold, st);
    } else if (dtype == DSMC_F32) {
        k_deflect<float><<<blocks, 256, 0, s>>>(n, (const float*)b, (const float*)g, (float*)chi,
                                                (float)hmk, P, q, gl, fold, st);
    } else {
        return arg_error("dsmc_deflect_jager: dtype %d", dtype);
    }
    DSMC_LAUNCH_CHECK("deflect_jager");
    return DSMC_OK;
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
        k_phaseA_jager<double><<<pb, 256, 0, s>>>(n_cells, pr, rng, v3<const double>(v), hmk,
                                                 b_max * 1e10, P, q, gl,
                                                 PairBuf<double>::of(ws, pairs.cap), st);
    } else {
        k_phaseA_jager<float><<<pb, 256, 0, s>>>(n_cells, pr, rng, v3<const float>(v), (float)hmk,
                                                (float)(b_max * 1e10), P, q, gl,
                                                PairBuf<float>::of(ws, pairs.cap), st);
    }
    DSMC_LAUNCH_CHECK("collide_jager:phaseA");
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
    return DSMC_OK;
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
        double c = chi_quad_wave<double>(P, q, gl, b, E, active);
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
