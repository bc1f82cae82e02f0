/*
 * CPU FP64 oracle for the DSMC collision step -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, sequential, obviously-correct reference for the GPU library.  Only
 * the tests, the smoke check and the benchmark's CPU-baseline leg may use it.
 * It shares no code with the GPU path.  Every function below names the part
 * of the paper (or the cited textbook method) it follows.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC dsmc_oracle.c
 */
#include "dsmc_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------
 * Philox4x32-10, from its published definition (Salmon et al., SC'11):
 * ten rounds of two 32x32->64 multiplies with the round constants below,
 * the key bumped by the Weyl increments between rounds.
 * ---------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void orc_draw(uint64_t seed, uint32_t step, uint32_t c0, uint32_t cell, uint32_t slot,
              uint32_t out[4])
{
    uint32_t ctr[4] = {c0, cell, step, slot};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* Uniform on [0,1) with 53 random bits: (a>>5)*2^26 + (b>>6), times 2^-53. */
static double u53(uint32_t a, uint32_t b)
{
    double hi = (double)(a >> 5);
    double lo = (double)(b >> 6);
    return (hi * 67108864.0 + lo) / 9007199254740992.0;
}

/* Uniform on [0,1) with 24 random bits. */
static double u24(uint32_t a)
{
    return (double)(a >> 8) / 16777216.0;
}

/* RNG slot numbers of the step's counter layout. */
enum { SLOT_CAND = 0, SLOT_COUNT = 1, SLOT_LAT0 = 2, SLOT_LAT1 = 3, SLOT_LAT2 = 4, SLOT_SBT = 5 };

/* ------------------------------------------------------------------------
 * Stable counting sort by cell id.
 * ---------------------------------------------------------------------- */
int orc_sort_cells(int32_t n, int32_t n_cells, const int32_t* cell_of,
                   int32_t* cell_start, int32_t* perm)
{
    int32_t* count = (int32_t*)calloc((size_t)n_cells + 1, sizeof(int32_t));
    int32_t bad = 0;
    for (int32_t p = 0; p < n; ++p) {
        int32_t c = cell_of[p];
        if (c < 0 || c >= n_cells) { ++bad; continue; }
        count[c] += 1;
    }
    cell_start[0] = 0;
    for (int32_t k = 0; k < n_cells; ++k) cell_start[k + 1] = cell_start[k] + count[k];
    /* cursor: next free slot of each cell, filled in original order (stable) */
    for (int32_t k = 0; k < n_cells; ++k) count[k] = cell_start[k];
    for (int32_t p = 0; p < n; ++p) {
        int32_t c = cell_of[p];
        if (c < 0 || c >= n_cells) continue;
        perm[count[c]] = p;
        count[c] += 1;
    }
    free(count);
    return bad;
}

/* ------------------------------------------------------------------------
 * Cell moments (section "Optional Cell-Wise Energy Drift Correction": the
 * per-cell energies E_pre/E_post; the centred sums S are the reading that
 * also restores momentum).  Sums run sequentially in sorted order.
 * ---------------------------------------------------------------------- */
static void cell_moments(int32_t s0, int32_t s1, const double* vx, const double* vy,
                         const double* vz, double out[6])
{
    int32_t N = s1 - s0;
    for (int q = 0; q < 6; ++q) out[q] = 0.0;
    if (N <= 0) return;
    double sx = 0, sy = 0, sz = 0;
    for (int32_t s = s0; s < s1; ++s) { sx += vx[s]; sy += vy[s]; sz += vz[s]; }
    double ux = sx / N, uy = sy / N, uz = sz / N;
    double S = 0, cmax = 0, E = 0;
    for (int32_t s = s0; s < s1; ++s) {
        double dx = vx[s] - ux, dy = vy[s] - uy, dz = vz[s] - uz;
        double c2 = dx * dx + dy * dy + dz * dz;
        S += c2;
        double c = sqrt(c2);
        if (c > cmax) cmax = c;
        E += vx[s] * vx[s] + vy[s] * vy[s] + vz[s] * vz[s];
    }
    out[0] = ux; out[1] = uy; out[2] = uz; out[3] = S; out[4] = cmax; out[5] = E;
}

void orc_moments(int32_t n_cells, const int32_t* cell_start, const double* vx,
                 const double* vy, const double* vz, double* mom)
{
    for (int32_t k = 0; k < n_cells; ++k)
        cell_moments(cell_start[k], cell_start[k + 1], vx, vy, vz, mom + 6 * (size_t)k);
}

/* ------------------------------------------------------------------------
 * NTC selection in one cell (section "Cell partition and collision-pair
 * selection"): the number of candidates is proportional to N(N-1) and to the
 * cell's upper bound (sigma g)_max; each candidate is a uniformly drawn
 * ordered pair i != j, accepted with probability sigma g / (sigma g)_max.
 *
 * Reading: (sigma g)_max uses g_hat = 2 max|c| (an exact bound on every pair's
 * g), the candidate count is rounded stochastically with one uniform, and the
 * acceptance test runs on the velocities as they were before the step.
 * Writes accepted local (i, j) in candidate order; returns the count.
 * ---------------------------------------------------------------------- */
static int32_t cell_candidates(int32_t N, double lam, double xs_C, double xs_e,
                               const double* mom_k, uint64_t seed, uint32_t step,
                               int32_t k)
{
    if (N < 2) return 0;
    double ghat = 2.0 * mom_k[4];
    double sgmax = xs_C * pow(ghat, xs_e);
    uint32_t r[4];
    orc_draw(seed, step, 0u, (uint32_t)k, SLOT_COUNT, r);
    double U = u53(r[0], r[1]);
    double x = 0.5 * (double)N * (double)(N - 1) * lam * sgmax + U;
    if (!(x >= 0.0) || !(x < 2147483647.0)) return 0;
    return (int32_t)floor(x);
}

static int32_t cell_select(int32_t s0, int32_t N, int32_t M, double xs_e, const double* mom_k,
                           const double* vx, const double* vy, const double* vz,
                           uint64_t seed, uint32_t step, int32_t k, int32_t* li,
                           int32_t* lj)
{
    double ghat = 2.0 * mom_k[4];
    int32_t acc = 0;
    for (int32_t t = 0; t < M; ++t) {
        uint32_t r[4];
        orc_draw(seed, step, (uint32_t)t, (uint32_t)k, SLOT_CAND, r);
        /* Lemire multiply-shift maps a 32-bit word to [0, N) without division */
        int32_t i = (int32_t)(((uint64_t)r[0] * (uint64_t)N) >> 32);
        int32_t j = (int32_t)(((uint64_t)r[1] * (uint64_t)(N - 1)) >> 32);
        if (j >= i) j += 1;
        double U = u53(r[2], r[3]);
        double dx = vx[s0 + i] - vx[s0 + j];
        double dy = vy[s0 + i] - vy[s0 + j];
        double dz = vz[s0 + i] - vz[s0 + j];
        double g = sqrt(dx * dx + dy * dy + dz * dz);
        double p = (xs_e == 1.0) ? g / ghat : pow(g / ghat, xs_e);
        if (U < p) {
            li[acc] = i;
            lj[acc] = j;
            ++acc;
        }
    }
    return acc;
}

int orc_select_ntc(int32_t n_cells, const int32_t* cell_start, const double* vx,
                   const double* vy, const double* vz, double xs_C, double xs_e,
                   const double* lambda, const double* mom, uint64_t seed,
                   uint32_t step, int32_t cell_base, int32_t* pair_off, int32_t* pair_cnt,
                   int32_t* pair_i, int32_t* pair_j, int32_t* pair_cell,
                   int64_t cap, int64_t* n_cand_total, int64_t* n_pairs_total)
{
    int64_t total = 0;
    for (int32_t k = 0; k < n_cells; ++k) {
        int32_t N = cell_start[k + 1] - cell_start[k];
        total += cell_candidates(N, lambda[k], xs_C, xs_e, mom + 6 * (size_t)k, seed, step,
                                 cell_base + k);
    }
    *n_cand_total = total;
    if (total > cap) {
        for (int32_t k = 0; k < n_cells; ++k) { pair_off[k] = 0; pair_cnt[k] = 0; }
        *n_pairs_total = 0;
        return 1;
    }
    int64_t np = 0;
    int32_t* li = NULL;
    int32_t* lj = NULL;
    int32_t lcap = 0;
    for (int32_t k = 0; k < n_cells; ++k) {
        int32_t s0 = cell_start[k], N = cell_start[k + 1] - s0;
        int32_t M = cell_candidates(N, lambda[k], xs_C, xs_e, mom + 6 * (size_t)k, seed, step,
                                    cell_base + k);
        if (M > lcap) {
            lcap = M;
            li = (int32_t*)realloc(li, sizeof(int32_t) * (size_t)lcap);
            lj = (int32_t*)realloc(lj, sizeof(int32_t) * (size_t)lcap);
        }
        int32_t a = cell_select(s0, N, M, xs_e, mom + 6 * (size_t)k, vx, vy, vz, seed, step,
                                cell_base + k, li, lj);
        pair_off[k] = (int32_t)np;
        pair_cnt[k] = a;
        for (int32_t q = 0; q < a; ++q) {
            pair_i[np + q] = s0 + li[q];
            pair_j[np + q] = s0 + lj[q];
            pair_cell[np + q] = k;
        }
        np += a;
    }
    free(li);
    free(lj);
    *n_pairs_total = np;
    return 0;
}

/* ------------------------------------------------------------------------
 * Simplified Bernoulli Trials (Stefanov 2011), the rate control the paper
 * names beside NTC: particle i (slot order, i = 0 .. N-2) gets one partner j
 * drawn uniformly from the m = N-1-i particles after it, and the pair
 * collides with probability m * lambda * sigma(g) g, so each unordered pair
 * {i, j} collides with probability lambda sigma(g_ij) g_ij -- the same
 * expectation as NTC.  Probabilities above 1 act as 1 and are counted.
 * ---------------------------------------------------------------------- */
int orc_select_sbt(int32_t n_cells, const int32_t* cell_start, const double* vx,
                   const double* vy, const double* vz, double xs_C, double xs_e,
                   const double* lambda, uint64_t seed, uint32_t step, int32_t cell_base,
                   int32_t* pair_off, int32_t* pair_cnt, int32_t* pair_i, int32_t* pair_j,
                   int32_t* pair_cell, int64_t cap, int64_t* n_trials_total,
                   int64_t* n_pairs_total, int32_t* n_clamped)
{
    int64_t total = 0;
    for (int32_t k = 0; k < n_cells; ++k) {
        int32_t N = cell_start[k + 1] - cell_start[k];
        if (N >= 2) total += N - 1;
    }
    *n_trials_total = total;
    *n_clamped = 0;
    if (total > cap) {
        for (int32_t k = 0; k < n_cells; ++k) { pair_off[k] = 0; pair_cnt[k] = 0; }
        *n_pairs_total = 0;
        return 1;
    }
    int64_t np = 0;
    for (int32_t k = 0; k < n_cells; ++k) {
        int32_t s0 = cell_start[k], N = cell_start[k + 1] - s0;
        int32_t a = 0;
        pair_off[k] = (int32_t)np;
        for (int32_t i = 0; i + 1 < N; ++i) {
            int32_t m = N - 1 - i;
            uint32_t r[4];
            orc_draw(seed, step, (uint32_t)i, (uint32_t)(cell_base + k), SLOT_SBT, r);
            int32_t j = i + 1 + (int32_t)(((uint64_t)r[0] * (uint64_t)m) >> 32);
            double U = u53(r[2], r[3]);
            double dx = vx[s0 + i] - vx[s0 + j];
            double dy = vy[s0 + i] - vy[s0 + j];
            double dz = vz[s0 + i] - vz[s0 + j];
            double g = sqrt(dx * dx + dy * dy + dz * dz);
            double sg = xs_C * ((xs_e == 1.0) ? g : pow(g, xs_e));
            double P = (double)m * lambda[k] * sg;
            if (P > 1.0) *n_clamped += 1;
            if (U < P) {
                pair_i[np + a] = s0 + i;
                pair_j[np + a] = s0 + j;
                pair_cell[np + a] = k;
                ++a;
            }
        }
        pair_cnt[k] = a;
        np += a;
    }
    *n_pairs_total = np;
    return 0;
}

/* ------------------------------------------------------------------------
 * Latents of one accepted pair (eq. mlp_input: xi ~ N(0, I3); plus the two
 * normals z that fix the impact parameter).  Normals by Box-Muller
 * (Box & Muller 1958) on pairs of uniforms; 1-U keeps the log argument in (0,1].
 * ---------------------------------------------------------------------- */
static void box_muller(double ua, double ub, double* n1, double* n2)
{
    double R = sqrt(-2.0 * log(1.0 - ua));
    double phi = 2.0 * ORC_PI * ub;
    *n1 = R * cos(phi);
    *n2 = R * sin(phi);
}

static void pair_uniforms(uint64_t seed, uint32_t step, uint32_t a, uint32_t k, int lowp,
                          double U[6])
{
    uint32_t r0[4], r1[4];
    orc_draw(seed, step, a, k, SLOT_LAT0, r0);
    orc_draw(seed, step, a, k, SLOT_LAT1, r1);
    if (lowp) {
        U[0] = u24(r0[0]); U[1] = u24(r0[1]); U[2] = u24(r0[2]); U[3] = u24(r0[3]);
        U[4] = u24(r1[0]); U[5] = u24(r1[1]);
    } else {
        uint32_t r2[4];
        orc_draw(seed, step, a, k, SLOT_LAT2, r2);
        U[0] = u53(r0[0], r0[1]); U[1] = u53(r0[2], r0[3]);
        U[2] = u53(r1[0], r1[1]); U[3] = u53(r1[2], r1[3]);
        U[4] = u53(r2[0], r2[1]); U[5] = u53(r2[2], r2[3]);
    }
}

static void latents_from_uniforms(const double U[6], double xi[3], double z[2])
{
    double spare;
    box_muller(U[0], U[1], &xi[0], &xi[1]);
    box_muller(U[2], U[3], &xi[2], &spare);
    box_muller(U[4], U[5], &z[0], &z[1]);
}

void orc_pair_latents(int64_t np, const int32_t* pair_cell, const int32_t* pair_off,
                      uint64_t seed, uint32_t step, int32_t cell_base, int lowp, double* U,
                      double* xi, double* z)
{
    for (int64_t p = 0; p < np; ++p) {
        int32_t k = pair_cell[p];
        uint32_t a = (uint32_t)(p - pair_off[k]);
        pair_uniforms(seed, step, a, (uint32_t)(cell_base + k), lowp, U + 6 * p);
        latents_from_uniforms(U + 6 * p, xi + 3 * p, z + 2 * p);
    }
}

/* Unit vector perpendicular to vhat along the component of xi orthogonal to
 * it (uniform azimuth, rotation invariant). */
static void perp_unit(const double xi[3], const double vh[3], double e[3])
{
    double d = xi[0] * vh[0] + xi[1] * vh[1] + xi[2] * vh[2];
    double w0 = xi[0] - d * vh[0], w1 = xi[1] - d * vh[1], w2 = xi[2] - d * vh[2];
    double n = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
    if (n > 0.0) {
        e[0] = w0 / n; e[1] = w1 / n; e[2] = w2 / n;
        return;
    }
    /* xi parallel to vhat: any perpendicular; take the cross product with the
       axis of vhat's smallest component */
    double ax = fabs(vh[0]), ay = fabs(vh[1]), az = fabs(vh[2]);
    double t[3] = {0, 0, 0};
    if (ax <= ay && ax <= az) t[0] = 1; else if (ay <= az) t[1] = 1; else t[2] = 1;
    w0 = vh[1] * t[2] - vh[2] * t[1];
    w1 = vh[2] * t[0] - vh[0] * t[2];
    w2 = vh[0] * t[1] - vh[1] * t[0];
    n = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
    e[0] = w0 / n; e[1] = w1 / n; e[2] = w2 / n;
}

static void unit_or_x(double a, double b, double c, double out[3], double* g)
{
    double n = sqrt(a * a + b * b + c * c);
    *g = n;
    if (n > 0.0) { out[0] = a / n; out[1] = b / n; out[2] = c / n; }
    else { out[0] = 1.0; out[1] = 0.0; out[2] = 0.0; }
}

/* Isotropic scattering (VHS/HS law): cos(chi) uniform on [-1, 1].  It is taken
 * as 2 btilde^2 - 1 with btilde^2 = 1 - exp(-|z|^2/2); for Box-Muller z that
 * quantity equals the uniform U[4] exactly, which is what is used, and
 * sin(chi) = sqrt((1-cos)(1+cos)) = 2 sqrt(U4 (1 - U4)). */
void orc_vhs_dirs(int64_t np, const int32_t* pair_i, const int32_t* pair_j,
                  const double* vx, const double* vy, const double* vz,
                  const double* U, const double* xi, double* u)
{
    for (int64_t p = 0; p < np; ++p) {
        int32_t a = pair_i[p], b = pair_j[p];
        double vh[3], g, e[3];
        unit_or_x(vx[a] - vx[b], vy[a] - vy[b], vz[a] - vz[b], vh, &g);
        double cc = 2.0 * U[6 * p + 4] - 1.0;
        double sc = 2.0 * sqrt(U[6 * p + 4] * (1.0 - U[6 * p + 4]));
        perp_unit(xi + 3 * p, vh, e);
        for (int q = 0; q < 3; ++q) u[3 * p + q] = cc * vh[q] + sc * e[q];
    }
}

/* Centre-of-mass pair update (eq. v_update_pair) with v_r' = g_current * u. */
static void apply_pair_dir(int32_t a, int32_t b, const double u[3], double* vx, double* vy,
                           double* vz)
{
    double rx = vx[a] - vx[b], ry = vy[a] - vy[b], rz = vz[a] - vz[b];
    double g = sqrt(rx * rx + ry * ry + rz * rz);
    double cx = 0.5 * (vx[a] + vx[b]), cy = 0.5 * (vy[a] + vy[b]), cz = 0.5 * (vz[a] + vz[b]);
    double px = g * u[0], py = g * u[1], pz = g * u[2];
    vx[a] = cx + 0.5 * px; vy[a] = cy + 0.5 * py; vz[a] = cz + 0.5 * pz;
    vx[b] = cx - 0.5 * px; vy[b] = cy - 0.5 * py; vz[b] = cz - 0.5 * pz;
}

void orc_apply_dirs(int32_t n_cells, const int32_t* pair_off, const int32_t* pair_cnt,
                    const int32_t* pair_i, const int32_t* pair_j, const double* u,
                    double* vx, double* vy, double* vz)
{
    for (int32_t k = 0; k < n_cells; ++k)
        for (int32_t q = 0; q < pair_cnt[k]; ++q) {
            int64_t p = (int64_t)pair_off[k] + q;
            apply_pair_dir(pair_i[p], pair_j[p], u + 3 * p, vx, vy, vz);
        }
}

static void apply_pair_chi(int32_t a, int32_t b, double cc, double sc, const double xi[3],
                           double* vx, double* vy, double* vz)
{
    double vh[3], g, e[3], d[3];
    unit_or_x(vx[a] - vx[b], vy[a] - vy[b], vz[a] - vz[b], vh, &g);
    perp_unit(xi, vh, e);
    for (int q = 0; q < 3; ++q) d[q] = cc * vh[q] + sc * e[q];
    apply_pair_dir(a, b, d, vx, vy, vz);
}

void orc_apply_chi(int32_t n_cells, const int32_t* pair_off, const int32_t* pair_cnt,
                   const int32_t* pair_i, const int32_t* pair_j, const double* cos_chi,
                   const double* sin_chi, const double* xi, double* vx, double* vy,
                   double* vz)
{
    for (int32_t k = 0; k < n_cells; ++k)
        for (int32_t q = 0; q < pair_cnt[k]; ++q) {
            int64_t p = (int64_t)pair_off[k] + q;
            apply_pair_chi(pair_i[p], pair_j[p], cos_chi[p], sin_chi[p], xi + 3 * p, vx, vy,
                           vz);
        }
}

/* ------------------------------------------------------------------------
 * Cell-wise moment matching (eq. cell_energy_clamp).  Centred reading: the
 * thermal energy S = sum|v-u|^2 is rescaled about the mean and the mean is
 * restored, v <- u_pre + alpha (v - u_post), alpha = sqrt(S_pre/S_post), so
 * both momentum and energy return to their pre-collision values.  Literal
 * reading: v <- alpha v with alpha = sqrt(E_pre/E_post).  Applied to cells
 * that had at least one collision and N >= 2, only if the post value is > 0.
 * ---------------------------------------------------------------------- */
static int cell_match(int32_t s0, int32_t s1, const double* mpre, int centred, double* vx,
                      double* vy, double* vz)
{
    double mpost[6];
    cell_moments(s0, s1, vx, vy, vz, mpost);
    if (centred) {
        double Spost = mpost[3];
        if (!(Spost > 0.0) || !isfinite(Spost)) return 1;
        double alpha = sqrt(mpre[3] / Spost);
        for (int32_t s = s0; s < s1; ++s) {
            vx[s] = mpre[0] + alpha * (vx[s] - mpost[0]);
            vy[s] = mpre[1] + alpha * (vy[s] - mpost[1]);
            vz[s] = mpre[2] + alpha * (vz[s] - mpost[2]);
        }
    } else {
        double Epost = mpost[5];
        if (!(Epost > 0.0) || !isfinite(Epost)) return 1;
        double alpha = sqrt(mpre[5] / Epost);
        for (int32_t s = s0; s < s1; ++s) {
            vx[s] *= alpha; vy[s] *= alpha; vz[s] *= alpha;
        }
    }
    return 0;
}

int32_t orc_moment_match(int32_t n_cells, const int32_t* cell_start,
                         const double* mom_pre, const int32_t* pair_cnt, int centred,
                         double* vx, double* vy, double* vz)
{
    int32_t skipped = 0;
    for (int32_t k = 0; k < n_cells; ++k) {
        int32_t s0 = cell_start[k], s1 = cell_start[k + 1];
        if (s1 - s0 < 2) continue;
        if (pair_cnt && pair_cnt[k] == 0) continue;
        skipped += cell_match(s0, s1, mom_pre + 6 * (size_t)k, centred, vx, vy, vz);
    }
    return skipped;
}

/* ------------------------------------------------------------------------
 * Potentials (section "The Jager ab initio Potential for Argon"):
 *   r >= 0.4 R_eps:  A exp(a1 r + a2 r^2 + a_-1/r + a_-2/r^2)
 *                    - sum_{n=3..8} f_2n(beta r) C_2n / r^2n
 *   r <  0.4 R_eps:  A_sr / r * exp(-a_sr r)
 * with the Tang-Toennies damping f_m(x) = 1 - exp(-x) sum_{k=0..m} x^k/k!
 * (eq. damping).  Hard sphere and inverse power are the closed-form checks.
 * ---------------------------------------------------------------------- */
static double tt_damping(int m, double x)
{
    double term = 1.0, sum = 0.0;
    for (int k = 0; k <= m; ++k) {
        sum += term;
        term = term * x / (double)(k + 1);
    }
    return 1.0 - exp(-x) * sum;
}

double orc_potential_V(const orc_potential* p, double r)
{
    if (!(r < 1e300)) return 0.0;
    switch (p->kind) {
    case ORC_POT_JAGER: {
        if (r < 0.4 * p->R_eps) return p->A_sr / r * exp(-p->a_sr * r);
        double rep = p->A * exp(p->a1 * r + p->a2 * r * r + p->am1 / r + p->am2 / (r * r));
        double disp = 0.0;
        for (int n = 3; n <= 8; ++n)
            disp += tt_damping(2 * n, p->beta_tt * r) * p->C[n - 3] / pow(r, 2 * n);
        return rep - disp;
    }
    case ORC_POT_HS:
        return (r < p->d) ? INFINITY : 0.0;
    case ORC_POT_INVPOW:
        return p->K / pow(r, p->n);
    }
    return NAN;
}

/* dV/dr, written out term by term; d/dx f_m(x) = exp(-x) x^m / m!. */
static double potential_dVdr(const orc_potential* p, double r)
{
    switch (p->kind) {
    case ORC_POT_JAGER: {
        if (r < 0.4 * p->R_eps) {
            double v = p->A_sr / r * exp(-p->a_sr * r);
            return -v * (p->a_sr + 1.0 / r);
        }
        double phi_r = p->a1 + 2.0 * p->a2 * r - p->am1 / (r * r) - 2.0 * p->am2 / (r * r * r);
        double rep = p->A * exp(p->a1 * r + p->a2 * r * r + p->am1 / r + p->am2 / (r * r));
        double dd = 0.0, x = p->beta_tt * r;
        for (int n = 3; n <= 8; ++n) {
            int m = 2 * n;
            double xm_over_mfact = 1.0;
            for (int k = 1; k <= m; ++k) xm_over_mfact *= x / (double)k;
            double fprime = exp(-x) * xm_over_mfact;
            double rm = pow(r, m);
            dd += p->C[n - 3] * (p->beta_tt * fprime / rm - m * tt_damping(m, x) / (rm * r));
        }
        return rep * phi_r - dd;
    }
    case ORC_POT_INVPOW:
        return -p->n * p->K / pow(r, p->n + 1);
    }
    return 0.0;
}

/* -int_a^{a+h} V'(r) dr by 3-point Gauss-Legendre. */
static double gauss3_minus_int_dV(const orc_potential* p, double a, double h)
{
    double half = 0.5 * h, mid = a + half, x = sqrt(0.6);
    return -half * ((5.0 / 9.0) * potential_dVdr(p, mid - half * x) +
                    (8.0 / 9.0) * potential_dVdr(p, mid) +
                    (5.0 / 9.0) * potential_dVdr(p, mid + half * x));
}

/* V(a) - V(a + h).  For |h| small against a the direct difference loses
 * digits, so it is taken as -int_a^{a+h} V'(r) dr by 3-point Gauss-Legendre,
 * whose error is far below rounding for |h| < 1e-3 a.  Passing the step h
 * itself (not a + h) keeps it exact.  The Jager form has two branches that
 * meet at 0.4 R_eps; a Gauss rule is exact only on one smooth branch, so an
 * interval that contains the meeting point is split there, and the
 * difference of the two branches at that point (V is continuous there only
 * to the accuracy of the coefficients) is added. */
double orc_potential_dV(const orc_potential* p, double a, double h)
{
    if (fabs(h) < 1e-3 * fabs(a)) {
        if (p->kind == ORC_POT_JAGER) {
            double rs = 0.4 * p->R_eps;
            if (h > 0.0 && a < rs && a + h > rs) {
                double inner = p->A_sr / rs * exp(-p->a_sr * rs);
                return gauss3_minus_int_dV(p, a, rs - a) + (inner - orc_potential_V(p, rs)) +
                       gauss3_minus_int_dV(p, rs, (a + h) - rs);
            }
        }
        return gauss3_minus_int_dV(p, a, h);
    }
    return orc_potential_V(p, a) - orc_potential_V(p, a + h);
}

typedef struct {
    const orc_potential* pot;
    double b, E;
    int64_t n_eval;
} chi_ctx;

/* D(r) = 1 - b^2/r^2 - V(r)/E: its largest zero is the distance of closest
 * approach r_min (the root equation of the "Exact" solver). */
static double D_of(chi_ctx* c, double r)
{
    c->n_eval += 1;
    return 1.0 - (c->b * c->b) / (r * r) - orc_potential_V(c->pot, r) / c->E;
}

/* Brent's method (Brent 1973, "Algorithms for Minimization without
 * Derivatives", ch. 4): bisection safeguarded inverse quadratic / secant
 * steps on a sign-changing bracket [a, b]. */
static double brent_root(chi_ctx* c, double a, double b, double fa, double fb)
{
    double cc = a, fc = fa, d = b - a, e = d;
    for (int it = 0; it < 200; ++it) {
        if ((fb > 0 && fc > 0) || (fb < 0 && fc < 0)) {
            cc = a; fc = fa; d = b - a; e = d;
        }
        if (fabs(fc) < fabs(fb)) {
            a = b; b = cc; cc = a;
            fa = fb; fb = fc; fc = fa;
        }
        double tol = 2.0 * DBL_EPSILON * fabs(b);
        double m = 0.5 * (cc - b);
        if (fabs(m) <= tol || fb == 0.0) return b;
        if (fabs(e) < tol || fabs(fa) <= fabs(fb)) {
            d = m; e = m;
        } else {
            double s = fb / fa, p, q;
            if (a == cc) {
                p = 2.0 * m * s;
                q = 1.0 - s;
            } else {
                double qq = fa / fc, r = fb / fc;
                p = s * (2.0 * m * qq * (qq - r) - (b - a) * (r - 1.0));
                q = (qq - 1.0) * (r - 1.0) * (s - 1.0);
            }
            if (p > 0) q = -q; else p = -p;
            double lim1 = 3.0 * m * q - fabs(tol * q), lim2 = fabs(e * q);
            if (2.0 * p < (lim1 < lim2 ? lim1 : lim2)) {
                e = d; d = p / q;
            } else {
                d = m; e = m;
            }
        }
        a = b; fa = fb;
        if (fabs(d) > tol) b += d;
        else b += (m > 0 ? tol : -tol);
        fb = D_of(c, b);
    }
    return b;
}

/* Largest zero of V (beyond it V < 0), needed to start the downward scan. */
static double jager_outer_zero(const orc_potential* p)
{
    double hi = 50.0, lo = hi;
    while (orc_potential_V(p, lo) <= 0.0 && lo > 1e-3) lo *= 0.99;
    for (int it = 0; it < 200; ++it) {
        double m = 0.5 * (lo + hi);
        if (orc_potential_V(p, m) > 0.0) lo = m; else hi = m;
    }
    return hi;
}

/* Gauss-Kronrod 7/15 nodes and weights on [-1, 1] (Kronrod extension of the
 * 7-point Gauss-Legendre rule, as tabulated in QUADPACK). */
static const double GK_X[8] = {
    0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
    0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
    0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
    0.207784955007898467600689403773245, 0.0};
static const double GK_WK[8] = {
    0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
    0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
    0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
    0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
static const double GK_WG[4] = {
    0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
    0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

typedef struct {
    chi_ctx* c;
    double rmin, beta, D0;
} integrand_ctx;

/* Integrand of the deflection integral after u = r_min/r (which maps the
 * range to [0,1]) and u = 1 - s^2 (which removes the inverse-square-root
 * endpoint singularity that remains at u = 1):
 *   chi = pi - 2 beta int_0^1 2 s / sqrt(F(1 - s^2)) ds,  beta = b / r_min,
 *   F(u) = beta^2 (1 - u^2) + (V(r_min) - V(r_min/u))/E + D0.
 * The potential difference is formed without cancellation (orc_potential_dV).
 * F is D(r_min/u) rewritten with D(r_min) = 0 taken exactly (D0 = 0) at a
 * smooth turning point; at a hard-sphere wall D0 = D(r_min+) = 1 - beta^2. */
static double integrand(integrand_ctx* q, double s)
{
    double s2 = s * s;
    double one_minus_u2 = s2 * (2.0 - s2);
    double dr = q->rmin * s2 / (1.0 - s2);  /* r - r_min with r = r_min / u */
    q->c->n_eval += 1;
    double dV = (q->c->pot->kind == ORC_POT_HS) ? 0.0
                                                : orc_potential_dV(q->c->pot, q->rmin, dr);
    double F = q->beta * q->beta * one_minus_u2 + dV / q->c->E + q->D0;
    if (!(F > 0.0)) return 0.0;  /* only reachable at s = 0 exactly */
    return 2.0 * s / sqrt(F);
}

static double gk15(integrand_ctx* q, double a, double b, double* err)
{
    double h = 0.5 * (b - a), mid = 0.5 * (a + b);
    double fc = integrand(q, mid);
    double k = fc * GK_WK[7], g = fc * GK_WG[3];
    for (int j = 0; j < 7; ++j) {
        double f1 = integrand(q, mid - h * GK_X[j]);
        double f2 = integrand(q, mid + h * GK_X[j]);
        k += GK_WK[j] * (f1 + f2);
        if (j % 2 == 1) g += GK_WG[j / 2] * (f1 + f2);
    }
    *err = fabs((k - g) * h);
    return k * h;
}

/* Globally adaptive bisection: the interval with the largest error estimate
 * is split until the summed estimate meets max(abs_tol, rel_tol |I|) or the
 * interval budget is spent (the scheme of QUADPACK's QAG, without its
 * extrapolation step, which the substitution above makes unnecessary). */
#define ADAPT_MAX 1024
#ifndef ADAPT_INIT
#define ADAPT_INIT 16
#endif
#ifndef ORC_QUAD_ABS
#define ORC_QUAD_ABS 1e-14
#endif
#ifndef ORC_QUAD_REL
#define ORC_QUAD_REL 1e-13
#endif
static double adapt(integrand_ctx* q, double a, double b, double abs_tol, double rel_tol)
{
    double lo[ADAPT_MAX], hi[ADAPT_MAX], val[ADAPT_MAX], err[ADAPT_MAX];
    /* start from ADAPT_INIT equal panels so that narrow interior peaks of the
       integrand (near-orbiting collisions) are sampled before adapting */
    int n = ADAPT_INIT;
    for (int j = 0; j < n; ++j) {
        lo[j] = a + (b - a) * j / n;
        hi[j] = (j == n - 1) ? b : a + (b - a) * (j + 1) / n;
        val[j] = gk15(q, lo[j], hi[j], &err[j]);
    }
    for (;;) {
        double I = 0.0, E = 0.0;
        int worst = 0;
        for (int j = 0; j < n; ++j) {
            I += val[j];
            E += err[j];
            if (err[j] > err[worst]) worst = j;
        }
        double tol = fmax(abs_tol, rel_tol * fabs(I));
        if (E <= tol || n >= ADAPT_MAX) return I;
        double m = 0.5 * (lo[worst] + hi[worst]);
        lo[n] = m; hi[n] = hi[worst];
        val[n] = gk15(q, m, hi[n], &err[n]);
        hi[worst] = m;
        val[worst] = gk15(q, lo[worst], m, &err[worst]);
        ++n;
    }
}

static double chi_impl(const orc_potential* pot, double b, double E, double r_zero,
                       int* status, int64_t* n_eval)
{
    chi_ctx c = {pot, b, E, 0};
    *status = 0;
    double rmin, D0 = 0.0;
    if (pot->kind == ORC_POT_HS) {
        rmin = b > pot->d ? b : pot->d;
        double beta = b / rmin;
        D0 = (b > pot->d) ? 0.0 : 1.0 - beta * beta;
    } else {
        double rhi;
        if (pot->kind == ORC_POT_JAGER) {
            rhi = b > r_zero ? b : r_zero;
        } else {
            if (!(pot->K >= 0.0)) { *status = 1; return NAN; }
            double rk = pow(2.0 * pot->K / E, 1.0 / pot->n);
            rhi = 2.0 * b > rk ? 2.0 * b : rk;
            if (!(rhi > 0.0)) rhi = 1.0;
        }
        double fhi = D_of(&c, rhi);
        if (fhi <= 0.0) {
            rmin = rhi;
        } else {
            /* downward geometric scan for the first sign change below rhi */
            double r = rhi, f = fhi, rl = rhi, fl = fhi;
            int found = 0;
            while (r > 1e-6) {
                rl = r * 0.999;
                fl = D_of(&c, rl);
                if (fl <= 0.0) { found = 1; break; }
                r = rl; f = fl;
            }
            if (!found) { *status = 1; if (n_eval) *n_eval = c.n_eval; return NAN; }
            rmin = (fl == 0.0) ? rl : brent_root(&c, rl, r, fl, f);
        }
    }
    double beta = b / rmin;
    integrand_ctx q = {&c, rmin, beta, D0};
    double I = adapt(&q, 0.0, 1.0, ORC_QUAD_ABS, ORC_QUAD_REL);
    if (n_eval) *n_eval = c.n_eval;
    return ORC_PI - 2.0 * beta * I;
}

double orc_chi(const orc_potential* p, double b, double E, int* status, int64_t* n_eval)
{
    double rz = (p->kind == ORC_POT_JAGER) ? jager_outer_zero(p) : 0.0;
    return chi_impl(p, b, E, rz, status, n_eval);
}

#define ORC_KB 1.380649e-23

void orc_chi_batch(const orc_potential* p, int64_t n, const double* b_m,
                   const double* g, double m_red, double* chi, int32_t* status,
                   int n_threads)
{
    double rz = (p->kind == ORC_POT_JAGER) ? jager_outer_zero(p) : 0.0;
#ifdef _OPENMP
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(n_threads)
#endif
    for (int64_t q = 0; q < n; ++q) {
        double E = 0.5 * m_red * g[q] * g[q] / ORC_KB; /* relative energy, K */
        int st;
        chi[q] = chi_impl(p, b_m[q] * 1e10, E, rz, &st, NULL);
        status[q] = st;
    }
}

/* ------------------------------------------------------------------------
 * Whole VHS collision step, cell by cell (parallel over cells, as the
 * section "Computational Framework" item 3 describes).
 * ---------------------------------------------------------------------- */
int64_t orc_step_vhs(int32_t n_cells, const int32_t* cell_start, double* vx,
                     double* vy, double* vz, double xs_C, double xs_e,
                     const double* lambda, uint64_t seed, uint32_t step,
                     int lowp, int moment_match, int n_threads)
{
    int64_t total = 0;
#ifdef _OPENMP
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel num_threads(n_threads) reduction(+ : total)
#endif
    {
        int32_t cap = 0;
        int32_t *li = NULL, *lj = NULL;
        double* dirs = NULL;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 8)
#endif
        for (int32_t k = 0; k < n_cells; ++k) {
            int32_t s0 = cell_start[k], N = cell_start[k + 1] - s0;
            double m[6];
            cell_moments(s0, s0 + N, vx, vy, vz, m);
            int32_t M = cell_candidates(N, lambda[k], xs_C, xs_e, m, seed, step, k);
            if (M > cap) {
                cap = M;
                li = (int32_t*)realloc(li, sizeof(int32_t) * (size_t)cap);
                lj = (int32_t*)realloc(lj, sizeof(int32_t) * (size_t)cap);
                dirs = (double*)realloc(dirs, sizeof(double) * 3 * (size_t)cap);
            }
            int32_t a = cell_select(s0, N, M, xs_e, m, vx, vy, vz, seed, step, k, li, lj);
            for (int32_t q = 0; q < a; ++q) {           /* Phase A: pre-step v */
                double U[6], xi[3], z[2], vh[3], g, e[3];
                pair_uniforms(seed, step, (uint32_t)q, (uint32_t)k, lowp, U);
                latents_from_uniforms(U, xi, z);
                int32_t ia = s0 + li[q], ib = s0 + lj[q];
                unit_or_x(vx[ia] - vx[ib], vy[ia] - vy[ib], vz[ia] - vz[ib], vh, &g);
                double cc = 2.0 * U[4] - 1.0, sc = 2.0 * sqrt(U[4] * (1.0 - U[4]));
                perp_unit(xi, vh, e);
                for (int d = 0; d < 3; ++d) dirs[3 * q + d] = cc * vh[d] + sc * e[d];
            }
            for (int32_t q = 0; q < a; ++q)            /* Phase B: in order */
                apply_pair_dir(s0 + li[q], s0 + lj[q], dirs + 3 * q, vx, vy, vz);
            if (moment_match && a > 0 && N >= 2) cell_match(s0, s0 + N, m, 1, vx, vy, vz);
            total += a;
        }
        free(li); free(lj); free(dirs);
    }
    return total;
}

/* ------------------------------------------------------------------------
 * Free flight, wall interaction and cell index: the DSMC move step around the
 * collision step (the flow cases of section "Results and Discussion": the
 * Couette channel between two diffuse walls and the lid-driven cavity with
 * diffuse walls).  The paper gives no formulas for this part; the standard
 * method (Bird 1994, ch. 11-12) is followed:
 *   - ballistic motion over dt, the earliest wall crossing handled first and
 *     the remaining time flown with the new velocity (at most ORC_MAX_HITS
 *     wall events per particle and step);
 *   - periodic sides shift the position by the period, specular sides flip
 *     the normal velocity, diffuse sides draw the velocity from the wall
 *     Maxwellian: normal component sigma_w sqrt(-2 ln(1 - U1)) (the flux
 *     weighted half-range Maxwellian), tangential components u_w + sigma_w n
 *     with n a Box-Muller pair of (U2, U3), sigma_w = sqrt(k T_w / m);
 *   - cell index ix = floor(x nx / Lx), clamped to the grid.
 * Random numbers: the wall event h of the particle in slot s draws
 * Philox(c0 = s, c1 = h, step, slot 6) -> (U1, U2) and (.., slot 7) -> U3,
 * 53-bit uniforms.  All arithmetic is FP64.
 * ---------------------------------------------------------------------- */
enum { SLOT_WALL0 = 6, SLOT_WALL1 = 7 };
#define ORC_MAX_HITS 8

static void wall_velocity(const orc_domain* dom, int side, uint64_t seed, uint32_t step,
                          uint32_t s, uint32_t h, double* vx, double* vy, double* vz)
{
    uint32_t r0[4], r1[4];
    orc_draw(seed, step, s, h, SLOT_WALL0, r0);
    orc_draw(seed, step, s, h, SLOT_WALL1, r1);
    const double U1 = u53(r0[0], r0[1]), U2 = u53(r0[2], r0[3]), U3 = u53(r1[0], r1[1]);
    const double sw = sqrt(ORC_KB * dom->T_w[side] / dom->m);
    const double vn = sw * sqrt(-2.0 * log(1.0 - U1));
    double n1, n2;
    box_muller(U2, U3, &n1, &n2);
    const double* uw = dom->u_w[side];
    /* sides 0/1: x = 0 / x = Lx (normal x); 2/3: y = 0 / y = Ly (normal y) */
    if (side < 2) {
        *vx = side == 0 ? vn : -vn;
        *vy = uw[1] + sw * n1;
        *vz = uw[2] + sw * n2;
    } else {
        *vy = side == 2 ? vn : -vn;
        *vx = uw[0] + sw * n1;
        *vz = uw[2] + sw * n2;
    }
}

int64_t orc_move(int32_t n, const orc_domain* dom, double dt, uint64_t seed, uint32_t step,
                 double* px, double* py, double* vx, double* vy, double* vz,
                 int32_t* cell_of, int64_t* n_hits)
{
    int64_t stuck = 0, hits = 0;
    const double Lx = dom->Lx, Ly = dom->Ly;
    for (int32_t s = 0; s < n; ++s) {
        double x = px[s], y = py[s], ux = vx[s], uy = vy[s], uz = vz[s];
        double t = dt;
        int h = 0;
        for (;;) {
            double tx = INFINITY, ty = INFINITY;
            if (ux > 0.0) tx = (Lx - x) / ux;
            else if (ux < 0.0) tx = -x / ux;
            if (uy > 0.0) ty = (Ly - y) / uy;
            else if (uy < 0.0) ty = -y / uy;
            if (tx >= t && ty >= t) {
                x = x + ux * t;
                y = y + uy * t;
                break;
            }
            if (h == ORC_MAX_HITS) {
                ++stuck;
                x = x + ux * t;
                y = y + uy * t;
                break;
            }
            int side;
            double th;
            if (tx <= ty) {
                side = ux > 0.0 ? 1 : 0;
                th = tx > 0.0 ? tx : 0.0;
                y = y + uy * th;
                x = side == 1 ? Lx : 0.0;
            } else {
                side = uy > 0.0 ? 3 : 2;
                th = ty > 0.0 ? ty : 0.0;
                x = x + ux * th;
                y = side == 3 ? Ly : 0.0;
            }
            t = t - th;
            const int kind = dom->kind[side];
            if (kind == ORC_WALL_PERIODIC) {
                if (side == 0) x = Lx;
                else if (side == 1) x = 0.0;
                else if (side == 2) y = Ly;
                else y = 0.0;
            } else if (kind == ORC_WALL_SPECULAR) {
                if (side < 2) ux = -ux; else uy = -uy;
            } else {
                wall_velocity(dom, side, seed, step, (uint32_t)s, (uint32_t)h, &ux, &uy, &uz);
            }
            ++h;
            ++hits;
        }
        /* keep the position inside the box (rounding at the walls) */
        if (x < 0.0) x = 0.0;
        if (x > Lx) x = Lx;
        if (y < 0.0) y = 0.0;
        if (y > Ly) y = Ly;
        px[s] = x; py[s] = y; vx[s] = ux; vy[s] = uy; vz[s] = uz;
        int32_t ix = (int32_t)(x * ((double)dom->nx / Lx));
        int32_t iy = (int32_t)(y * ((double)dom->ny / Ly));
        ix = ix < 0 ? 0 : (ix >= dom->nx ? dom->nx - 1 : ix);
        iy = iy < 0 ? 0 : (iy >= dom->ny ? dom->ny - 1 : iy);
        cell_of[s] = iy * dom->nx + ix;
    }
    if (n_hits) *n_hits = hits;
    return stuck;
}

/* ------------------------------------------------------------------------
 * Cell sampling for the macroscopic fields (velocity, temperature, shear
 * stress and heat flux of the flow results): per cell, raw moment sums
 * acc[13k + ...] += (1, vx, vy, vz, vx^2, vy^2, vz^2, vx vy, vx vz, vy vz,
 * |v|^2 vx, |v|^2 vy, |v|^2 vz), in slot order.
 * ---------------------------------------------------------------------- */
void orc_sample(int32_t n_cells, const int32_t* cell_start, const double* vx,
                const double* vy, const double* vz, double* acc)
{
    for (int32_t k = 0; k < n_cells; ++k) {
        double* a = acc + 13 * (size_t)k;
        for (int32_t s = cell_start[k]; s < cell_start[k + 1]; ++s) {
            const double x = vx[s], y = vy[s], z = vz[s];
            const double e = x * x + y * y + z * z;
            a[0] += 1.0;
            a[1] += x; a[2] += y; a[3] += z;
            a[4] += x * x; a[5] += y * y; a[6] += z * z;
            a[7] += x * y; a[8] += x * z; a[9] += y * z;
            a[10] += e * x; a[11] += e * y; a[12] += e * z;
        }
    }
}
