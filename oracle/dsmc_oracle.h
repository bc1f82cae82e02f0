/*
 * CPU FP64 oracle for the DSMC collision step -- TEST INFRASTRUCTURE ONLY.
 *
 * This is the plain, slow reference that the GPU library is checked against.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product path never does.  It shares no code with
 * the GPU library: its Philox generator, sort, selection, scattering rules,
 * root finder and quadrature are all written here independently.
 *
 * Everything works on SoA velocity arrays (vx, vy, vz) in cell-sorted order,
 * with cell k owning sorted slots [cell_start[k], cell_start[k+1]).
 */
#ifndef DSMC_ORACLE_H
#define DSMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Draw for the step's counter layout: ctr = (c0, cell, step, slot), key = seed. */
void orc_draw(uint64_t seed, uint32_t step, uint32_t c0, uint32_t cell, uint32_t slot,
              uint32_t out[4]);

/* Stable counting sort of particles by cell (section "Computational Framework",
 * item 1: particles sorted by cell index, contiguous per cell). */
int orc_sort_cells(int32_t n, int32_t n_cells, const int32_t* cell_of,
                   int32_t* cell_start, int32_t* perm);

/* Per-cell moments: mom[6k..6k+5] = (ux, uy, uz, S, cmax, E) with
 * u = mean velocity, S = sum |v-u|^2, cmax = max |v-u|, E = sum |v|^2
 * (E is the cell energy of the cell-wise clamp equation). */
void orc_moments(int32_t n_cells, const int32_t* cell_start, const double* vx,
                 const double* vy, const double* vz, double* mom);

/* NTC selection (section "Cell partition and collision-pair selection").
 * sigma*g = xs_C * g^xs_e.  Cell k of the arrays is global cell cell_base + k
 * (the id that keys the random numbers), so a contiguous range of cells can
 * be checked on its own.  Returns 0, or 1 on pair-capacity overflow (then
 * *n_cand_total holds the required capacity and no pair is written). */
int orc_select_ntc(int32_t n_cells, const int32_t* cell_start, const double* vx,
                   const double* vy, const double* vz, double xs_C, double xs_e,
                   const double* lambda, const double* mom, uint64_t seed,
                   uint32_t step, int32_t cell_base, int32_t* pair_off, int32_t* pair_cnt,
                   int32_t* pair_i, int32_t* pair_j, int32_t* pair_cell,
                   int64_t cap, int64_t* n_cand_total, int64_t* n_pairs_total);
int orc_select_sbt(int32_t n_cells, const int32_t* cell_start, const double* vx,
                   const double* vy, const double* vz, double xs_C, double xs_e,
                   const double* lambda, uint64_t seed, uint32_t step, int32_t cell_base,
                   int32_t* pair_off, int32_t* pair_cnt, int32_t* pair_i, int32_t* pair_j,
                   int32_t* pair_cell, int64_t cap, int64_t* n_trials_total,
                   int64_t* n_pairs_total, int32_t* n_clamped);

/* Per-pair latent draws.  U[6p..6p+5] uniforms, xi[3p..] and z[2p..] normals.
 * lowp = 1 selects the 24-bit uniform construction used for FP32 velocities. */
void orc_pair_latents(int64_t np, const int32_t* pair_cell, const int32_t* pair_off,
                      uint64_t seed, uint32_t step, int32_t cell_base, int lowp, double* U,
                      double* xi, double* z);

/* Isotropic (VHS/HS) post-collision direction from pre-step velocities. */
void orc_vhs_dirs(int64_t np, const int32_t* pair_i, const int32_t* pair_j,
                  const double* vx, const double* vy, const double* vz,
                  const double* U, const double* xi, double* u);

/* Phase B: in-cell ordered application of per-pair unit directions u. */
void orc_apply_dirs(int32_t n_cells, const int32_t* pair_off, const int32_t* pair_cnt,
                    const int32_t* pair_i, const int32_t* pair_j, const double* u,
                    double* vx, double* vy, double* vz);

/* Phase B for deflection angles: rotate the current v_r by chi about the
 * azimuth direction that xi defines. */
void orc_apply_chi(int32_t n_cells, const int32_t* pair_off, const int32_t* pair_cnt,
                   const int32_t* pair_i, const int32_t* pair_j, const double* cos_chi,
                   const double* sin_chi, const double* xi, double* vx, double* vy,
                   double* vz);

/* Cell-wise moment matching after the collisions (eq. cell_energy_clamp);
 * centred = 1: momentum-and-energy form, 0: the literal lab-frame rescale.
 * Returns the number of cells skipped. */
int32_t orc_moment_match(int32_t n_cells, const int32_t* cell_start,
                         const double* mom_pre, const int32_t* pair_cnt, int centred,
                         double* vx, double* vy, double* vz);

/* Interaction potentials.  r in Angstrom, V/k_B in K. */
enum { ORC_POT_JAGER = 0, ORC_POT_HS = 1, ORC_POT_INVPOW = 2 };
typedef struct {
    int32_t kind;
    int32_t n;          /* INVPOW exponent */
    double A, a1, a2, am1, am2, beta_tt;
    double C[6];        /* C6..C16 */
    double R_eps, A_sr, a_sr;
    double d;           /* HS diameter */
    double K;           /* INVPOW strength */
} orc_potential;

double orc_potential_V(const orc_potential* p, double r);
/* V(a) - V(a + h) without cancellation for small h. */
double orc_potential_dV(const orc_potential* p, double a, double h);

/* Deflection angle chi(b, E) of the classical deflection integral, with
 * b in Angstrom and E/k_B in K.  *status: 0 ok, 1 root not found.
 * n_eval (nullable) receives the number of potential evaluations. */
double orc_chi(const orc_potential* p, double b, double E, int* status, int64_t* n_eval);

/* Batch version over SI inputs (b in m, g in m/s, reduced mass in kg). */
void orc_chi_batch(const orc_potential* p, int64_t n, const double* b_m,
                   const double* g, double m_red, double* chi, int32_t* status,
                   int n_threads);

/* Whole collision step with the VHS rule (select, Phase A, Phase B, optional
 * moment match) on sorted arrays; used for CPU timing.  Returns #pairs. */
int64_t orc_step_vhs(int32_t n_cells, const int32_t* cell_start, double* vx,
                     double* vy, double* vz, double xs_C, double xs_e,
                     const double* lambda, uint64_t seed, uint32_t step,
                     int lowp, int moment_match, int n_threads);

/* Domain of the move step: nx x ny uniform cells over [0, Lx] x [0, Ly];
 * sides 0..3 = x = 0, x = Lx, y = 0, y = Ly, each periodic, specular or
 * diffuse (wall temperature T_w, wall velocity u_w); m = particle mass. */
enum { ORC_WALL_PERIODIC = 0, ORC_WALL_SPECULAR = 1, ORC_WALL_DIFFUSE = 2 };
typedef struct {
    int32_t nx, ny;
    double Lx, Ly;
    int32_t kind[4];
    double T_w[4];
    double u_w[4][3];
    double m;
} orc_domain;

/* Move step: free flight over dt with wall events; positions and velocities
 * updated in place, cell_of[n] written.  Returns the number of particles that
 * reached the wall-event limit; *n_hits = wall events. */
int64_t orc_move(int32_t n, const orc_domain* dom, double dt, uint64_t seed, uint32_t step,
                 double* px, double* py, double* vx, double* vy, double* vz,
                 int32_t* cell_of, int64_t* n_hits);

/* Raw per-cell moment sums for the macroscopic fields (13 per cell,
 * accumulated into acc). */
void orc_sample(int32_t n_cells, const int32_t* cell_start, const double* vx,
                const double* vy, const double* vz, double* acc);

#ifdef __cplusplus
}
#endif
#endif
