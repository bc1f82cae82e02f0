// Per-pair arithmetic of the ab initio deflection angle (section
// "Computational Implementation: The Exact vs. Neural Paradigm"), written once
// for the device kernels and for host-side set-up:
//
//   chi(b, E) = pi - 2 b int_{r_min}^inf dr / (r^2 sqrt(D(r))),
//   D(r) = 1 - b^2/r^2 - V(r)/E,  r_min = the largest root of D.
//
// u = r_min / r maps the range to [0, 1] and u = 1 - t^2 removes the
// inverse-square-root singularity left at u = 1, so
//   chi = pi - 2 beta int_0^1 2 t / sqrt(F(t)) dt,  beta = b / r_min,
//   F(t) = beta^2 t^2 (2 - t^2) + (V(r_min) - V(r))/E = D(r(t)),
//   r(t) = r_min / (1 - t^2).
//
// Two levels:
//  * chi_lane: one lane per pair in the kernel's precision T.  Root by a
//    downward geometric scan (with a check at every local minimum of the
//    sampled D, so a narrow negative dip of D is never stepped over) and
//    safeguarded Newton; the integral by one fixed Gauss-Legendre rule in t.
//    Pairs for which this is not accurate -- a sharp peak of the integrand
//    near orbiting, where F comes close to zero inside the range (a positive
//    local minimum of D above r_min) or at t = 0 (D'(r_min) small) -- or
//    whose root is uncertain are flagged.
//  * the refinement (FP64): a 64-point geometric scan of D in parallel, the
//    local minimum of D and the root polished by safeguarded iterations, and
//    the integral with the sinh substitution t = c + w sinh(s) centred on the
//    peak (Johnston & Elliott, "A sinh transformation for evaluating nearly
//    singular boundary element integrals", 2005): with F ~ F* + k (t - c)^2
//    near the peak and w = sqrt(F*/k), the transformed integrand is nearly
//    constant there, so one Gauss-Legendre rule per side of the peak
//    converges.  The kernels spread its samples and nodes over a wavefront.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/dsmc.h"

#define CQ_HD __host__ __device__ __forceinline__

namespace dsmc {

constexpr int GL_MAX = 128;

struct GLRule {
    int n;
    double t[GL_MAX];  // nodes on [0, 1]
    double w[GL_MAX];  // weights on [0, 1] (sum 1)
};

// Potential and the set-up quantities the quadrature needs.
struct Pot {
    dsmc_potential p;
    double r_sw;     // short-range switch 0.4 R_eps (JAGER)
    double r_zero;   // largest zero of V (JAGER); V < 0 beyond it
    double e_scan;   // below this E (K) D may have several roots (orbiting)
    double r_floor;  // below e_scan every root of D lies above this radius
    double v_jump;   // V(r_sw-) - V(r_sw+): mismatch of the JAGER branches
};

struct QuadCfg {
    int max_iter;     // root iterations
    int refine;       // 1: flagged pairs get the FP64 refinement
    double scan_ratio;  // geometric step of the lane's low-energy scan
};

// Number of samples of the refinement's parallel scan (one per lane), and
// Gauss-Legendre panels per side of the mapped peak (equal in s).
constexpr int REF_SAMPLES = 64;
constexpr int REF_PANELS = 2;

// ------------------------------------------------------------------------
// Potential (T arithmetic)
// ------------------------------------------------------------------------
// Damped dispersion sum of the JAGER form, sum_n f_n(x) C_n r^-n over
// n = 6, 8, ..., 16 with x = beta_tt r and the Tang-Toennies factors
// f_n(x) = 1 - e^-x sum_{k<=n} x^k/k!, and (DERIV) its r-derivative, using
// f_n'(x) = e^-x x^n/n!.  Beyond x = 60 every f_n is 1 to better than 1e-13
// (and x^16 would overflow FP32).  Where f_n is small (x well below n) the
// difference 1 - e^-x S_n cancels; in FP32 below x = 8 the factors are
// summed from the series tail instead, f_n = sum_{k>n} e^-x x^k/k!,
// downward from n = 16 (positive terms only; the tail of f_16 is summed to
// k = 40, where (8/18)^23 is far below FP32 rounding).
constexpr double DAMP_OFF = 60.0;
constexpr double TAIL_X = 8.0;

template <typename T> CQ_HD T cq_exp(T x) { return exp(x); }
template <> CQ_HD float cq_exp<float>(float x) { return expf(x); }

template <typename T, bool DERIV>
CQ_HD void tt_disp(const dsmc_potential& p, T r, T ri, T& disp, T& ddisp)
{
    const T x = T(p.beta_tt) * r;
    const T ri2 = ri * ri;
    disp = T(0);
    ddisp = T(0);
    if (x >= T(DAMP_OFF)) {
        T rpow = ri2 * ri2 * ri2;  // r^-6
#pragma unroll
        for (int n = 0; n < 6; ++n) {
            disp += T(p.C[n]) * rpow;
            if (DERIV) ddisp -= T(6 + 2 * n) * T(p.C[n]) * rpow * ri;
            rpow *= ri2;
        }
        return;
    }
    const T ex = cq_exp<T>(-x);
    if (sizeof(T) < sizeof(double) && x < T(TAIL_X)) {
        // (loops kept rolled: this branch is rare and must not raise the
        // register count of the common one)
        T e = ex;  // e_k = e^-x x^k / k!
#pragma unroll 1
        for (int k = 1; k <= 16; ++k) e = e * x / T(k);
        T f = T(0), ek = e;
#pragma unroll 1
        for (int k = 17; k <= 40; ++k) {
            ek = ek * x / T(k);
            f += ek;
        }
        const T r2 = r * r, xi = T(1) / x;
        T r8 = ri2 * ri2;
        r8 = r8 * r8;
        T rpow = r8 * r8;  // r^-16
#pragma unroll 1
        for (int n = 5; n >= 0; --n) {
            const int m = 6 + 2 * n;  // f = f_m, e = e_m
            disp += f * T(p.C[n]) * rpow;
            if (DERIV) ddisp += T(p.C[n]) * (T(p.beta_tt) * e * rpow - T(m) * f * rpow * ri);
            const T e1 = e * T(m) * xi;         // e_{m-1}
            const T e2 = e1 * T(m - 1) * xi;    // e_{m-2}
            f += e + e1;                        // f_{m-2}
            e = e2;
            rpow *= r2;
        }
        return;
    }
    T term = T(1), S = T(1);
    T rpow = ri2 * ri2 * ri2;
#pragma unroll
    for (int k = 1; k <= 16; ++k) {
        term = term * x * T(1.0 / k);  // x^k / k!
        S += term;
        if (k >= 6 && (k & 1) == 0) {
            const T C = T(p.C[(k - 6) / 2]);
            const T f = T(1) - ex * S;
            disp += f * C * rpow;
            if (DERIV) ddisp += C * (T(p.beta_tt) * ex * term * rpow - T(k) * f * rpow * ri);
            rpow *= ri2;
        }
    }
}

// V(r) and, with DERIV, V'(r) from one evaluation of the shared factors.
template <typename T, bool DERIV>
CQ_HD T pot_eval(const Pot& P, T r, T& dV)
{
    const dsmc_potential& p = P.p;
    if (p.kind == DSMC_POT_INVPOW) {
        T rn = r;
        for (int q = 1; q < p.n; ++q) rn *= r;
        const T V = T(p.K) / rn;
        dV = -T(p.n) * V / r;
        return V;
    }
    const T ri = T(1) / r;
    if (r < T(P.r_sw)) {
        const T V = T(p.A_sr) * ri * cq_exp<T>(-T(p.a_sr) * r);
        dV = -V * (T(p.a_sr) + ri);
        return V;
    }
    const T rep = T(p.A) * cq_exp<T>(T(p.a1) * r + T(p.a2) * r * r + T(p.am1) * ri + T(p.am2) * ri * ri);
    T disp, ddisp;
    tt_disp<T, DERIV>(p, r, ri, disp, ddisp);
    if (DERIV) {
        const T phi_r = T(p.a1) + T(2) * T(p.a2) * r - T(p.am1) * ri * ri - T(2) * T(p.am2) * ri * ri * ri;
        dV = rep * phi_r - ddisp;
    }
    return rep - disp;
}

template <typename T>
CQ_HD T V_of(const Pot& P, T r)
{
    T unused;
    return pot_eval<T, false>(P, r, unused);
}

template <typename T>
CQ_HD T dV_of(const Pot& P, T r)
{
    T dV;
    pot_eval<T, true>(P, r, dV);
    return dV;
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

// D(r) = 1 - b^2/r^2 - V(r)/E and its derivative.
template <typename T>
CQ_HD T D_of(const Pot& P, T b2, T E, T r)
{
    return T(1) - b2 / (r * r) - V_of<T>(P, r) / E;
}
template <typename T>
CQ_HD T dD_of(const Pot& P, T b2, T E, T r)
{
    return T(2) * b2 / (r * r * r) - dV_of<T>(P, r) / E;
}

// One value of the t integrand, 2 t / sqrt(F) with
// F = beta^2 t^2 (2 - t^2) + (V(r_min) - V(r))/E + D0 and r = r_min / (1 - t^2);
// also F / t^2 (the peak indicator: r_min D'(r_min) at t = 0, 1 at t = 1).
// Near r_min the potential difference is -int V' dr by 2-point
// Gauss-Legendre (no cancellation).  F <= 0 (only possible if r_min is not
// the largest root) counts in *nonpos.
template <typename T>
CQ_HD T node_term(const Pot& P, T rmin, T beta, T Vmin, T E, T D0, T t, T& f_over_t2, int& nonpos)
{
    const T g1 = T(0.5) - T(0.28867513459481287);
    const T g2 = T(0.5) + T(0.28867513459481287);
    const T t2 = t * t;
    const T dr = rmin * t2 / (T(1) - t2);
    T dV = T(0);
    if (P.p.kind != DSMC_POT_HS) {
        if (t2 < T(1e-3)) {
            const T rs = T(P.r_sw);
            if (rmin < rs && rmin + dr > rs) {
                // the two branches of the JAGER form meet inside the step:
                // integrate each side on its own, plus the (set-up) jump
                const T h1 = rs - rmin, h2 = rmin + dr - rs;
                dV = -h1 * T(0.5) * (dV_of<T>(P, rmin + g1 * h1) + dV_of<T>(P, rmin + g2 * h1)) -
                     h2 * T(0.5) * (dV_of<T>(P, rs + g1 * h2) + dV_of<T>(P, rs + g2 * h2)) +
                     T(P.v_jump);
            } else {
                dV = -dr * T(0.5) * (dV_of<T>(P, rmin + g1 * dr) + dV_of<T>(P, rmin + g2 * dr));
            }
        } else {
            dV = Vmin - V_of<T>(P, rmin + dr);
        }
    }
    const T F = beta * beta * t2 * (T(2) - t2) + dV / E + D0;
    f_over_t2 = F / t2;
    if (F > T(0)) return T(2) * t / sqrt(F);
    nonpos += 1;
    return T(0);
}

// Gauss-Legendre over t in [ta, tb]; qmin tracks min F / t^2 over the nodes.
template <typename T>
CQ_HD T integral_part(const Pot& P, const GLRule& gl, T rmin, T beta, T Vmin, T E, T D0, T ta,
                      T tb, T& qmin, int& nonpos)
{
    const T len = tb - ta;
    T I = T(0);
    for (int k = 0; k < gl.n; ++k) {
        T fq;
        I += T(gl.w[k]) * node_term<T>(P, rmin, beta, Vmin, E, D0, ta + len * T(gl.t[k]), fq, nonpos);
        qmin = fq < qmin ? fq : qmin;
    }
    return len * I;
}

// Safeguarded Newton for a root of D in [rlo, rhi] with D(rlo) <= 0 < D(rhi),
// starting from r0; returns the root and D' there.
template <typename T>
CQ_HD T root_newton(const Pot& P, int max_iter, T b2, T E, T rlo, T rhi, T r0, T& dD)
{
    T r = r0;
    dD = T(0);
    for (int it = 0; it < max_iter; ++it) {
        T dV;
        const T V = pot_eval<T, true>(P, r, dV);
        const T f = T(1) - b2 / (r * r) - V / E;
        if (f > T(0)) rhi = r; else rlo = r;
        const T fp = T(2) * b2 / (r * r * r) - dV / E;
        dD = fp;
        T rn = r - f / fp;
        if (!(rn > rlo && rn < rhi)) rn = T(0.5) * (rlo + rhi);
        const T step = rn - r;
        r = rn;
        if (fabs(step) <= Consts<T>::rtol * r || rhi - rlo <= Consts<T>::rtol * r) break;
    }
    return r;
}

// Lane-level flag thresholds.
//  Q0_FLAG: r_min D'(r_min) below this marks an endpoint peak (t = 0).
//  QN_FLAG: min of F / t^2 over the rule's nodes below this marks a peak.
//  W_FLAG:  estimated half-width (in t) of an interior peak below this.
//  DM_MARGIN: a local minimum of the sampled D whose parabola estimate is
//    below this may hide a negative dip: the root is left to the refinement.
//  Q0_HIGH: r_min D'(r_min) above this (|V|/E of tens to thousands, a few K
//    and below) marks an integrand whose dynamic range one rule of n nodes
//    does not resolve to the precision's bound.
// The values were set by comparing unflagged pairs with the oracle over the
// deflection batch, a batch of relative speeds 10-400 m/s and the Mach-10
// cylinder's pairs: FP64 stays below 1e-9 rad and FP32 below 6e-5 rad while
// 2 % (FP64) and 0.4-1.8 % (FP32) of the pairs are flagged.
template <typename T> struct LaneTol;
template <> struct LaneTol<double> {
    static constexpr double Q0_FLAG = 0.05, QN_FLAG = 0.2, W_FLAG = 0.1, DM_MARGIN = 0.02, Q0_HIGH = 250.0;
};
template <> struct LaneTol<float> {
    static constexpr float Q0_FLAG = 0.3f, QN_FLAG = 0.3f, W_FLAG = 0.1f, DM_MARGIN = 0.05f, Q0_HIGH = 500.0f;
};

// chi(b, E) with b in Angstrom, E/k_B in K, in the lane's precision.  NaN if
// the root search failed.  *flag: the pair needs the FP64 refinement.
// diag (optional): receives the flag indicators r_min D'(r_min), the node
// minimum of F / t^2 and the interior peak half-width estimate.
template <typename T>
CQ_HD T chi_lane(const Pot& P, const QuadCfg& q, const GLRule& gl, double bd, double Ed, bool& flag,
                 T* diag = nullptr)
{
    const T pi = Consts<T>::pi;
    const T b = T(bd), E = T(Ed);
    const T b2 = b * b;
    flag = false;
    T rmin, D0 = T(0), dD = T(0);
    const bool jager = P.p.kind == DSMC_POT_JAGER;
    const bool low = jager && E < T(P.e_scan);
    T w_int = T(1e30);  // interior peak half-width estimate
    if (P.p.kind == DSMC_POT_HS) {
        const T d = T(P.p.d);
        rmin = b > d ? b : d;
        const T beta = b / rmin;
        D0 = b > d ? T(0) : T(1) - beta * beta;
    } else {
        T rhi;
        if (jager) {
            rhi = b > T(P.r_zero) ? b : T(P.r_zero);
        } else {
            const T rk = pow(T(2) * T(P.p.K) / E, T(1) / T(P.p.n));
            rhi = T(2) * b > rk ? T(2) * b : rk;
            if (!(rhi > T(0))) rhi = T(1);
        }
        T f1 = D_of<T>(P, b2, E, rhi);
        if (f1 <= T(0)) {
            rmin = rhi;
            if (low) flag = true;
        } else {
            const T ratio = low ? T(q.scan_ratio) : T(0.7);
            T r1 = rhi, r0 = T(-1), f0 = T(0), rlo = T(0), r_start = T(0);
            bool found = false, have_min = false;
            T pk_rm = T(0), pk_dm = T(0), pk_d2 = T(0);
            for (int it = 0; it < 4000; ++it) {
                const T r2 = r1 * ratio;
                const T f2 = D_of<T>(P, b2, E, r2);
                if (f2 <= T(0)) {
                    rlo = r2;
                    rhi = r1;
                    r_start = (-f2 < f1) ? r2 : r1;
                    found = true;
                    break;
                }
                if (low && r0 > T(0) && f1 < f0 && f1 < f2) {
                    // The samples passed a local minimum of D inside
                    // (r2, r0): parabola through the three samples (in r).
                    const T h0 = r0 - r1, h2 = r1 - r2;
                    const T s0 = (f0 - f1) / h0, s2 = (f1 - f2) / h2;
                    const T d2 = T(2) * (s0 - s2) / (h0 + h2);  // D''
                    const T d1 = s2 + T(0.5) * d2 * h2;          // D'(r1)
                    const T dm = f1 - T(0.5) * d1 * d1 / d2;     // minimum value
                    if (!(dm > T(LaneTol<T>::DM_MARGIN)) || !(d2 > T(0))) {
                        flag = true;  // a dip may reach zero: refinement
                        return T(0);
                    }
                    // A positive minimum: the root is the inner one, on the
                    // repulsive side of the well.  The scan started at b, so
                    // b > r_zero and D(r_zero) = 1 - b^2/r_zero^2 < 0.
                    have_min = true;
                    pk_rm = r1 - d1 / d2;
                    pk_dm = dm;
                    pk_d2 = d2;
                    rlo = T(P.r_zero);
                    rhi = r2;
                    r_start = T(P.r_zero);
                    found = true;
                    break;
                }
                r0 = r1;
                f0 = f1;
                r1 = r2;
                f1 = f2;
                if (r2 < T(1e-4)) break;
            }
            if (!found) {
                if (low) flag = true;
                return T(NAN);
            }
            rmin = root_newton<T>(P, q.max_iter, b2, E, rlo, rhi, r_start, dD);
            if (have_min) {
                // interior peak of the integrand at t* = sqrt(1 - r_min/r_m):
                // F ~ D(r_m) + D''(r_m) r'(t*)^2 (t - t*)^2 / 2 with
                // r' = 2 r_min t* / (1 - t*^2)^2
                const T ts2 = T(1) - rmin / pk_rm;
                const T ts = ts2 > T(0) ? sqrt(ts2) : T(0);
                const T om = T(1) - ts2;
                const T rp = T(2) * rmin * ts / (om * om);
                w_int = sqrt(T(2) * pk_dm / (pk_d2 * rp * rp + T(1e-30)));
            }
        }
    }
    T beta = b / rmin;
    T Vmin = (P.p.kind == DSMC_POT_HS) ? T(0) : V_of<T>(P, rmin);
    if (sizeof(T) < sizeof(double) && low) {
        // FP32 below the orbiting energy: |V|/E reaches ~10 and V(r_min) is
        // the difference of repulsive and dispersion terms ~70 E apart, so
        // an FP32 root and V(r_min) would offset F by ~1e-5.  One FP64
        // Newton step from the FP32 root, rounded to FP32 (the nodes map
        // from that point), then V(r_min) and beta in FP64 there: r_min is
        // the exact turning point of a problem with 1 - D(r_min) ~ 1e-8 in
        // place of 1.  F's other terms stay FP32; a root that moves is left
        // to the refinement.  (Loop kept rolled: one inlined evaluation.)
        const double b2d = bd * bd, r0 = double(rmin);
        double r = r0, Vd = 0.0;
#pragma unroll 1
        for (int it = 0; it < 2; ++it) {
            double dVd;
            Vd = pot_eval<double, true>(P, r, dVd);
            if (it == 1) break;
            r -= (1.0 - b2d / (r * r) - Vd / Ed) / (2.0 * b2d / (r * r * r) - dVd / Ed);
            if (!(fabs(r - r0) <= 1e-5 * r)) flag = true;
            r = double(T(r));
        }
        rmin = T(r);
        beta = T(bd / r);
        Vmin = T(Vd);
    }
    T I = T(0);
    T qmin = T(1e30);
    int nonpos = 0;
    if (low) {
        // low energy: r_min lies outside the short-range region
        I = integral_part<T>(P, gl, rmin, beta, Vmin, E, D0, T(0), T(1), qmin, nonpos);
        const T q0 = rmin * dD;
        if (diag) {
            diag[0] = q0;
            diag[1] = qmin;
            diag[2] = w_int;
        }
        if (q0 < T(LaneTol<T>::Q0_FLAG) || q0 > T(LaneTol<T>::Q0_HIGH) ||
            qmin < T(LaneTol<T>::QN_FLAG) || w_int < T(LaneTol<T>::W_FLAG) || nonpos > 0)
            flag = true;
    } else {
        // the short-range switch of the JAGER form is a kink of the
        // integrand: integrate the two sides separately
        T tsw = T(1);
        if (jager && rmin < T(P.r_sw)) tsw = sqrt(T(1) - rmin / T(P.r_sw));
        I = integral_part<T>(P, gl, rmin, beta, Vmin, E, D0, T(0), tsw, qmin, nonpos);
        if (tsw < T(1)) I += integral_part<T>(P, gl, rmin, beta, Vmin, E, D0, tsw, T(1), qmin, nonpos);
    }
    return pi - T(2) * beta * I;
}

// ------------------------------------------------------------------------
// FP64 refinement pieces (uniform across the wave that runs them)
// ------------------------------------------------------------------------
struct RefState {
    double b2, E;
    double rmin, beta, Vmin;
    double c, w;          // peak centre and half-width in t (w = 0: no map)
    double s_lo, s_hi;    // s range of the two sides: [s_lo, 0] and [0, s_hi]
    int sides;            // 1: right side only (c = 0); 2: both
    int ok;
};

// Sample grid of the parallel scan: r_k = rtop * rho^k, k = 0..63, from
// max(b, r_zero) down past r_floor.
CQ_HD void ref_grid(const Pot& P, double b, double& rtop, double& rho)
{
    rtop = b > P.r_zero ? b : P.r_zero;
    const double rbot = 0.98 * P.r_floor;
    rho = exp(log(rbot / rtop) / (REF_SAMPLES - 1));
}
CQ_HD double ref_sample_r(double rtop, double rho, int k)
{
    return rtop * exp(k * log(rho));
}

// Parallel bracketing: in each round the 64 lanes evaluate a function at
// x_l = a + (b - a) l / 63 (both ends included) and the bracket becomes
// [x_{L-1}, x_L] around the first lane L whose value is positive, so each
// round narrows it 63-fold at the cost of one evaluation per lane.  The
// callers bracket D' around the local minimum of D (negative below r_m) and
// D around the root (negative below r_min), REF_ROUNDS rounds each, then
// take the secant through the final bracket.
constexpr int REF_ROUNDS = 4;
CQ_HD double ref_x(double a, double b, int l) { return l == 63 ? b : a + (b - a) * (l * (1.0 / 63.0)); }
CQ_HD int ref_pick(int first_pos) { return first_pos < 1 ? 1 : (first_pos > 63 ? 63 : first_pos); }

// Sets the sinh map of the integral once r_min (and beta, V(r_min)) are in
// s: around the interior minimum of F at r_m (D(r_m) = dm > 0, D''(r_m) =
// d2m) if there is one, else around t = 0 where F / t^2 ~ Q0 + Q2 t^2 with
// Q0 = r_min D'(r_min) and Q2 = Q0 + D''(r_min) r_min^2 / 2.
CQ_HD void ref_map(RefState& s, bool has_min, double rm, double dm, double d2m, double dD,
                   double d2D)
{
    double c = 0.0, w = 0.0;
    if (has_min && dm > 0.0 && rm > s.rmin) {
        // interior peak at t* = sqrt(1 - r_min / r_m): F ~ dm + d2m r'^2 (t - t*)^2 / 2
        // with r' = 2 r_min t* / (1 - t*^2)^2
        const double ts2 = 1.0 - s.rmin / rm;
        c = sqrt(ts2);
        const double om = 1.0 - ts2;
        const double rp = 2.0 * s.rmin * c / (om * om);
        const double k = 0.5 * d2m * rp * rp;
        w = k > 0.0 ? sqrt(dm / k) : 1.0;
    } else {
        const double q0 = s.rmin * dD;
        const double q2 = q0 + 0.5 * d2D * s.rmin * s.rmin;
        w = (q0 > 0.0 && q2 > 0.0) ? sqrt(q0 / q2) : 1.0;
    }
    if (!(w > 1e-12)) w = 1e-12;
    if (w > 1.0) w = 1.0;
    s.c = c;
    s.w = w;
    s.sides = c > 0.0 ? 2 : 1;
    s.s_lo = c > 0.0 ? asinh(-c / w) : 0.0;
    s.s_hi = asinh((1.0 - c) / w);
}

// Weighted integrand at node m (0 <= m < ref_nodes(s, gl)) of the mapped rule:
// REF_PANELS equal panels in s on each side of the peak.
CQ_HD int ref_nodes(const RefState& s, const GLRule& gl) { return s.sides * REF_PANELS * gl.n; }
CQ_HD double ref_node(const Pot& P, const GLRule& gl, const RefState& s, int m, int& nonpos)
{
    const int seg = m / gl.n, j = m - seg * gl.n;
    const int side = (s.sides == 2) ? seg / REF_PANELS : 1;
    const int pnl = seg % REF_PANELS;
    const double a = side ? 0.0 : s.s_lo, bnd = side ? s.s_hi : 0.0;
    const double len = (bnd - a) / REF_PANELS;
    const double sv = a + len * (pnl + gl.t[j]);
    const double t = s.c + s.w * sinh(sv);
    double fq;
    return gl.w[j] * len * s.w * cosh(sv) *
           node_term<double>(P, s.rmin, s.beta, s.Vmin, s.E, 0.0, t, fq, nonpos);
}

// ------------------------------------------------------------------------
// Host-side set-up: Gauss-Legendre nodes, potential constants, settings.
// ------------------------------------------------------------------------
int arg_error(const char* fmt, ...);

// Gauss-Legendre nodes by Newton on P_n (mapped to [0, 1]).
inline int make_gl(int n, GLRule* g)
{
    if (n == 0) n = 64;
    if (n < 2 || n > GL_MAX) return arg_error("dsmc_quad: n_nodes %d not in [2, %d]", n, GL_MAX);
    g->n = n;
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double x = cos(pi * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                const double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            const double dp = n * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; ++k) {
            const double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = pk;
        }
        const double dp = n * (x * p1 - p0) / (x * x - 1.0);
        g->t[i] = 0.5 * (1.0 - x);
        g->w[i] = 1.0 / ((1.0 - x * x) * dp * dp);  // (2 / ((1-x^2) P'^2)) / 2
    }
    return DSMC_OK;
}

inline int make_pot(const dsmc_potential* pot, Pot* P)
{
    if (!pot) return arg_error("dsmc potential: null");
    P->p = *pot;
    P->r_sw = 0.0;
    P->r_zero = 0.0;
    P->e_scan = 0.0;
    P->r_floor = 0.0;
    P->v_jump = 0.0;
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
        P->v_jump = pot->A_sr / P->r_sw * exp(-pot->a_sr * P->r_sw) - V_of<double>(*P, P->r_sw);
        // largest zero of V: scan in from 50 A, then bisect
        double hi = 50.0, lo = 50.0;
        while (V_of<double>(*P, lo) <= 0.0 && lo > 0.05) lo *= 0.99;
        if (V_of<double>(*P, lo) <= 0.0) return arg_error("dsmc potential: V has no repulsive core");
        for (int it = 0; it < 200; ++it) {
            const double m = 0.5 * (lo + hi);
            if (V_of<double>(*P, m) > 0.0) lo = m; else hi = m;
        }
        P->r_zero = hi;
        // Energy above which r^2 (1 - V(r)/E) is increasing in r on the
        // outer region (one turning point for every b); below it D can have
        // three roots.  Found on a grid, then doubled for margin.
        double ecrit = 0.0;
        for (double E = 1.0; E < 1e5; E *= 1.05) {
            bool mono = true;
            double prev = -1e300;
            for (double r = 0.6 * P->r_zero; r < 40.0; r *= 1.002) {
                const double B = r * r * (1.0 - V_of<double>(*P, r) / E);
                if (B < prev) { mono = false; break; }
                prev = B;
            }
            if (mono) { ecrit = E; break; }
        }
        P->e_scan = ecrit > 0 ? 2.0 * ecrit : 1e30;
        // Below e_scan a root r of D has V(r) = E (1 - b^2/r^2) <= E < e_scan,
        // and V decreases monotonically inside r_zero: every root lies above
        // the radius where V = e_scan.
        double a = 1e-3, c = P->r_zero;
        for (int it = 0; it < 200; ++it) {
            const double m = 0.5 * (a + c);
            if (V_of<double>(*P, m) > P->e_scan) a = m; else c = m;
        }
        P->r_floor = a;
        return DSMC_OK;
    }
    }
    return arg_error("dsmc potential: kind %d", pot->kind);
}

inline int make_cfg(const dsmc_quad& q, QuadCfg* c, GLRule* gl)
{
    c->max_iter = q.max_iter > 0 ? q.max_iter : 60;
    c->scan_ratio = q.scan_ratio > 0 ? q.scan_ratio : 0.95;
    c->refine = q.refine >= 0 ? 1 : 0;
    if (!(c->scan_ratio > 0.5 && c->scan_ratio < 1.0))
        return arg_error("dsmc_quad: scan_ratio %g not in (0.5, 1)", c->scan_ratio);
    return make_gl(q.n_nodes, gl);
}

}  // namespace dsmc
