/*
 * dsmc.h -- C-ABI of the MI355X (gfx950) DSMC collision-step library.
 *
 * The library implements the collision step of Direct Simulation Monte Carlo
 * as the paper (Roohi, Shoja-sani, Stefanov, arXiv 2602.21244) states it in
 * section "DSMC collision step and scope of replacement": particles are sorted
 * into cells, candidate pairs are selected per cell by the No-Time-Counter
 * scheme, and each accepted pair's post-collision relative velocity comes from
 * a scattering rule -- the isotropic VHS law, the ab initio deflection angle
 * chi(b, g) by quadrature of the classical deflection integral, or the paper's
 * neural surrogate (conditional MLP with latent noise, energy-shell projection)
 * -- followed by cell-wise moment matching.
 *
 * Conventions (all entry points):
 *  - Every array argument is a caller-owned DEVICE pointer unless it says
 *    "host".  The library never allocates or frees caller memory; scratch
 *    memory is a caller-owned workspace whose size the *_ws query returns.
 *  - Every call is asynchronous on the given HIP stream (NULL = the default
 *    stream), performs no host synchronisation and no allocation, and can be
 *    captured into a HIP graph.  Data-dependent outcomes (pair counts,
 *    overflow, root-search failures) are written to a caller-owned device
 *    status word, never returned to the host.
 *  - Return value: DSMC_OK, or a negative code for errors detectable on the
 *    host (null pointers, bad enums or sizes: DSMC_E_ARG; a failed launch:
 *    DSMC_E_HIP; a shape without a compiled kernel: DSMC_E_UNSUPPORTED).
 *    dsmc_last_error() returns a thread-local message for the last error.
 *  - Velocities are structure-of-arrays (vx, vy, vz), FP64 or FP32, in m/s.
 *    After dsmc_sort_cells they are in cell-sorted order: cell k owns sorted
 *    slots [cell_start[k], cell_start[k+1]).
 *  - Randomness is counter-based Philox4x32-10 keyed by (seed) with counter
 *    (index, cell, step, slot), so results do not depend on launch shape or
 *    schedule and are reproducible bit for bit.
 */
#ifndef DSMC_H
#define DSMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* dsmc_stream_t; /* hipStream_t */

enum { DSMC_OK = 0, DSMC_E_ARG = -1, DSMC_E_HIP = -2, DSMC_E_UNSUPPORTED = -3 };
enum { DSMC_F32 = 0, DSMC_F64 = 1, DSMC_BF16 = 2 };

/* SoA velocity components (device arrays of the chosen dtype). */
typedef struct { void* x; void* y; void* z; } dsmc_vec3;

/* Philox key and step counter of one collision step. */
typedef struct { uint64_t seed; uint32_t step; uint32_t reserved; } dsmc_rng;

/* Device status word (caller-owned device memory).  Counters accumulate
 * across calls until dsmc_status_clear. */
typedef struct {
    uint32_t flags;     /* DSMC_ST_* bits */
    int32_t bad_cell;   /* particles whose cell id was outside [0, n_cells) */
    int64_t n_cand;     /* candidates of the last selection (capacity needed) */
    int64_t n_pairs;    /* accepted pairs of the last selection */
    int32_t root_fail;  /* deflection evaluations whose root search failed */
    int32_t nonfinite;  /* non-finite values met (results left unchanged) */
    int32_t mm_skipped; /* cells that moment matching left alone (S_post <= 0) */
    int32_t prob_clamped; /* SBT trials whose collision probability exceeded 1 */
    int64_t wall_events;  /* wall crossings handled by dsmc_move */
    int32_t wall_limit;   /* particles that met the wall-event limit of one move */
    int32_t reserved;
} dsmc_status;
enum {
    DSMC_ST_PAIR_OVERFLOW = 1u, /* candidates exceeded the pair capacity */
    DSMC_ST_BAD_CELL = 2u,
    DSMC_ST_ROOT_FAIL = 4u,
    DSMC_ST_NONFINITE = 8u,
    DSMC_ST_PROB_CLAMP = 16u,   /* an SBT probability exceeded 1 (time step too large) */
    DSMC_ST_WALL_LIMIT = 32u    /* a particle met 8 wall events in one move */
};

/* Accepted-pair list, dense and cell-major: the pairs of cell k are entries
 * [off[k], off[k] + cnt[k]) in candidate order.  i and j are sorted slots. */
typedef struct {
    int32_t* off;  /* [n_cells] */
    int32_t* cnt;  /* [n_cells] */
    int32_t* i;    /* [cap] */
    int32_t* j;    /* [cap] */
    int32_t* cell; /* [cap] owning cell of each pair */
    int64_t cap;   /* capacity of i, j, cell -- and the most candidates a
                      selection may draw (more sets DSMC_ST_PAIR_OVERFLOW) */
} dsmc_pairs;

/* Cross-section law of the selection stage (kept unchanged by the paper):
 * VHS sigma_T(g) = pi d_ref^2 (2 k T_ref/(m_r g^2))^(omega-1/2) / Gamma(5/2-omega),
 * m_r = m/2 (Bird 1994); CONST: sigma (the paper's constant reference cross
 * section).  All SI units. */
enum { DSMC_XS_VHS = 0, DSMC_XS_CONST = 1 };
typedef struct {
    int32_t kind;
    int32_t reserved;
    double m, d_ref, omega, T_ref; /* VHS */
    double sigma;                  /* CONST */
} dsmc_xs;

/* Interaction potential for the deflection angle.  r in Angstrom, V/k_B in K.
 * JAGER: the paper's modified Tang-Toennies form (eq. jager_potential with the
 *   damping of eq. damping) for r >= 0.4 R_eps, screened Coulomb A_sr/r
 *   exp(-a_sr r) below.  C[] = C6..C16; beta_tt is the damping constant.
 * HS: hard sphere of diameter d.  INVPOW: V = K / r^n (n = 1..12). */
enum { DSMC_POT_JAGER = 0, DSMC_POT_HS = 1, DSMC_POT_INVPOW = 2 };
typedef struct {
    int32_t kind;
    int32_t n;
    double A, a1, a2, am1, am2, beta_tt;
    double C[6];
    double R_eps, A_sr, a_sr;
    double d;
    double K;
} dsmc_potential;

/* Quadrature settings of the deflection integral.  n_nodes: Gauss-Legendre
 * nodes per panel (8..128; 0 = 64).  scan_ratio: geometric step of the
 * downward root scan below the energy at which D can have several roots
 * (0 = 0.95; every local minimum the scan passes is checked, so a narrow
 * negative dip of D is not stepped over).  max_iter: root refinement
 * iterations (0 = 60).  refine: >= 0 (default): pairs whose integrand has a
 * sharp peak near orbiting, or whose root is uncertain, are re-evaluated in
 * FP64 by the whole wavefront (parallel root scan, polished local minimum
 * and root, sinh substitution centred on the peak); -1: off, every pair
 * keeps the one-rule result (for accuracy and timing comparison). */
typedef struct {
    int32_t n_nodes;
    int32_t max_iter;
    double scan_ratio;
    int32_t refine;
    int32_t reserved;
} dsmc_quad;

/* Conditional MLP f_theta (section "Cell-Based Neural Collision Operator"):
 * h_l = act(W_l h_{l-1} + b_l) for hidden layers, linear output layer.
 * W[l] is row-major [dims[l+1]][dims[l]].  wdtype DSMC_BF16: W in bf16, b in
 * fp32, MFMA path (every hidden width 64, 128 or 256, dims[0] <= 30,
 * dims[L] <= 32, and the weights in fragment order within the 160 KB LDS of
 * a CU: any depth at width 64, up to five hidden layers at 128, one at 256;
 * other shapes return DSMC_E_UNSUPPORTED).  wdtype DSMC_F64: W, b in fp64, FP64 reference path (any
 * width up to 256).  The input row is x = [v_r/sigma_v (3), xi (3), z (2)]
 * (eq. mlp_input plus the two impact latents), so dims[0] must be 8 for the
 * in-step entry point. */
enum { DSMC_ACT_SILU = 0, DSMC_ACT_RELU = 1 };
/* How activations enter the matrix cores on the bf16 path (dsmc_mlp.split).
 * DSMC_SPLIT_ALL (0, the default of a zeroed struct): the network input and
 * every hidden activation as a bf16 pair hi + lo (16 significant bits); the
 * result is that of the bf16 weights to ~1e-4 rad in direction.
 * DSMC_SPLIT_FRONT: the input and the first two hidden activations as pairs,
 * later hidden activations as one bf16 value: about a sixth fewer matrix
 * operations and conversions, at a direction error of a few 1e-3 rad for a
 * trained 8-128x4-3 network (rounding early in the network is amplified
 * most).  DSMC_SPLIT_FIRST: the input and the first hidden activation only
 * (a third fewer pair operations than FRONT, about twice its direction
 * error).  Applies to dsmc_neural_collide; the row entry points always use
 * DSMC_SPLIT_ALL. */
enum { DSMC_SPLIT_ALL = 0, DSMC_SPLIT_FRONT = 1, DSMC_SPLIT_FIRST = 2 };
typedef struct {
    int32_t n_layers;
    int32_t dims[7];
    int32_t act;
    int32_t wdtype;
    const void* W[6];
    const void* b[6];
    double sigma_v;
    int32_t split;
    int32_t reserved;
} dsmc_mlp;

/* Phase-B schedules: LANE: one lane walks a cell's pairs in order; WAVE: one
 * wavefront per cell, velocities staged in LDS, applying in rounds every
 * pending pair that is the earliest pending pair of both its particles
 * (cells of up to 256 pairs spanning up to 1024 particles); BLOCK: the same
 * rounds by a 256-lane workgroup on global memory (any cell).  AUTO: LANE
 * up to an autotuned pair count, WAVE above it, BLOCK for cells WAVE cannot
 * hold.  All schedules give bit-identical results. */
enum { DSMC_SCHED_AUTO = 0, DSMC_SCHED_LANE = 1, DSMC_SCHED_BLOCK = 2, DSMC_SCHED_WAVE = 4 };
/* DSMC_SCHED_DEFER: run Phase A only and leave its per-pair results in the
 * workspace; dsmc_apply_pairs then performs Phase B (used to overlap or time
 * the two phases separately). */
enum { DSMC_SCHED_DEFER = 3 };
/* Phase-A result kinds for dsmc_apply_pairs. */
enum { DSMC_APPLY_DIRECTIONS = 0, DSMC_APPLY_ANGLES = 1 };

/* Moment-matching modes (eq. cell_energy_clamp). */
enum { DSMC_MM_CAPTURE = 0, DSMC_MM_APPLY = 1, DSMC_MM_APPLY_LITERAL = 2 };

/* ---------------------------------------------------------------------- */

/* Select the device used by later calls from this thread (hipSetDevice);
 * optional. */
int dsmc_init(int device);
const char* dsmc_last_error(void);
const char* dsmc_version(void);

/* Zero the status word on the stream (a fill kernel, graph-safe). */
int dsmc_status_clear(dsmc_status* st, dsmc_stream_t stream);

/* Bin particles into cells (section "Computational Framework", item 1:
 * particles sorted by cell index so each cell is contiguous).
 * Stable sort by cell_of[n] (original order kept inside a cell; a radix
 * sort of the cell ids): writes cell_start[n_cells+1] (exclusive prefix of
 * the counts), perm[n] (perm[s] = original index of sorted slot s) and
 * gathers v_in into v_out (distinct buffers).  Ids outside [0, n_cells) are
 * counted in st->bad_cell and sorted after every kept particle: then
 * cell_start[n_cells] < n and slots cell_start[n_cells]..n-1 hold the dropped
 * particles in original order.  n_cells < 2^31 - 1.
 * ws: dsmc_sort_cells_ws(n, n_cells) bytes (about 12 n + 4 KiB per 4096
 * particles, plus a few bytes per thousand cells for the count scan). */
size_t dsmc_sort_cells_ws(int32_t n, int32_t n_cells);
int dsmc_sort_cells(int32_t n, int32_t n_cells, const int32_t* cell_of, int32_t dtype,
                    dsmc_vec3 v_in, dsmc_vec3 v_out, int32_t* cell_start, int32_t* perm,
                    void* ws, size_t ws_bytes, dsmc_status* st, dsmc_stream_t stream);

/* dsmc_sort_cells without a workspace, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same results, bit for bit, with the
 * scratch in a static device array of the library (about 14 MB, one copy per
 * GPU, held until the process ends).  Limits: n <= 1 048 576 particles and
 * n_cells <= 1 048 576; larger inputs return DSMC_E_ARG (use
 * dsmc_sort_cells).  The call allocates nothing (no hipMalloc/hipFree, no
 * allocating library routine).  All calls on one GPU share the array:
 * calls that overlap on one GPU (concurrent streams or threads) race. */
int dsmc_sort_cells_noalloc(int32_t n, int32_t n_cells, const int32_t* cell_of, int32_t dtype,
                            dsmc_vec3 v_in, dsmc_vec3 v_out, int32_t* cell_start, int32_t* perm,
                            dsmc_status* st, dsmc_stream_t stream);

/* Cell moments and cell-wise moment matching (section "Optional Cell-Wise
 * Energy Drift Correction", eq. cell_energy_clamp), FP64 throughout.
 * mom[6*n_cells] per cell: (ux, uy, uz, S, cmax, E) with u the mean velocity,
 * S = sum |v-u|^2, cmax = max |v-u|, E = sum |v|^2.
 * CAPTURE: write mom from v.  APPLY: for every cell with N >= 2 and (if
 * pair_cnt is not NULL) pair_cnt[k] > 0, set v <- u_pre + alpha (v - u_post),
 * alpha = sqrt(S_pre / S_post): restores the cell's momentum and energy.
 * APPLY_LITERAL: v <- alpha v with alpha = sqrt(E_pre / E_post) (the
 * equation as printed; conserves energy only).  Cells with a non-positive or
 * non-finite post value are left unchanged and counted in st->mm_skipped. */
int dsmc_moment_match(int32_t n_cells, const int32_t* cell_start, int32_t dtype,
                      dsmc_vec3 v, double* mom, int32_t mode, const int32_t* pair_cnt,
                      dsmc_status* st, dsmc_stream_t stream);

/* No-Time-Counter pair selection (section "Cell partition and
 * collision-pair selection"): per cell with N >= 2 particles,
 *   M = floor(N (N-1)/2 * lambda_k * (sigma g)_max + U),
 * (sigma g)_max from g_hat = 2 cmax (mom from CAPTURE, an exact bound on the
 * cell's pair speeds); each candidate t draws an ordered pair i != j
 * uniformly and is accepted iff U_t < sigma(g) g / (sigma g)_max, on the
 * velocities as passed (pre-collision).  lambda[n_cells] = F_N dt / V_c.
 * If the total candidate count exceeds pairs.cap no pair is written,
 * DSMC_ST_PAIR_OVERFLOW is set and st->n_cand holds the capacity needed.
 * ws: dsmc_select_pairs_ntc_ws(n_cells, cap) bytes. */
size_t dsmc_select_pairs_ntc_ws(int32_t n_cells, int64_t cap);
int dsmc_select_pairs_ntc(int32_t n_cells, const int32_t* cell_start, int32_t dtype,
                          dsmc_vec3 v, dsmc_xs xs, const double* lambda, const double* mom,
                          dsmc_rng rng, dsmc_pairs pairs, void* ws, size_t ws_bytes,
                          dsmc_status* st, dsmc_stream_t stream);

/* Simplified Bernoulli Trials selection (Stefanov 2011), the alternative rate
 * control the paper names beside NTC (section "Cell partition and
 * collision-pair selection"): per cell with N >= 2, trial t = 0 .. N-2 takes
 * the particle in slot t, draws its partner uniformly among the m = N-1-t
 * later slots (Philox slot 5, Lemire multiply-shift) and accepts with
 * probability P = m lambda_k sigma(g) g on the velocities as passed
 * (P > 1 acts as 1; counted in st->prob_clamped with DSMC_ST_PROB_CLAMP).
 * Same pair-list output as dsmc_select_pairs_ntc (trial order = candidate
 * order); expected pairs per cell lambda_k sum_{i<j} sigma g_ij, as NTC.
 * More than pairs.cap trials: nothing written, DSMC_ST_PAIR_OVERFLOW.
 * ws: dsmc_select_pairs_sbt_ws(n_cells, cap) bytes. */
size_t dsmc_select_pairs_sbt_ws(int32_t n_cells, int64_t cap);
int dsmc_select_pairs_sbt(int32_t n_cells, const int32_t* cell_start, int32_t dtype,
                          dsmc_vec3 v, dsmc_xs xs, const double* lambda, dsmc_rng rng,
                          dsmc_pairs pairs, void* ws, size_t ws_bytes, dsmc_status* st,
                          dsmc_stream_t stream);

/* Workspace of the collide entry points below (per-pair Phase-A results). */
size_t dsmc_collide_ws(int64_t cap, int32_t dtype);

/* Isotropic VHS scattering (the plain rule the paper replaces; isotropy
 * check of section "Generalization Test"): Phase A per accepted pair on the
 * pre-collision velocities -- cos chi uniform on [-1,1], azimuth from the
 * latent xi -- then Phase B per cell in candidate order on the current
 * velocities: v_r' = |v_r| u, v_i = v_cm + v_r'/2, v_j = v_cm - v_r'/2
 * (eq. v_update_pair).  Exactly conserves each pair's momentum and energy. */
int dsmc_collide_vhs(int32_t n_cells, int32_t dtype, dsmc_vec3 v, dsmc_pairs pairs,
                     dsmc_rng rng, int32_t schedule, void* ws, size_t ws_bytes,
                     dsmc_stream_t stream);

/* Phase B alone, from the Phase-A results a collide call left in `ws` with
 * schedule DSMC_SCHED_DEFER: kind DSMC_APPLY_DIRECTIONS after
 * dsmc_collide_vhs / dsmc_neural_collide, DSMC_APPLY_ANGLES after
 * dsmc_collide_jager.  schedule: AUTO, LANE or BLOCK. */
int dsmc_apply_pairs(int32_t n_cells, int32_t dtype, dsmc_vec3 v, dsmc_pairs pairs, int32_t kind,
                     int32_t schedule, void* ws, size_t ws_bytes, dsmc_stream_t stream);

/* Phase B fused with the cell-wise moment matching (section "Optional
 * Cell-Wise Energy Drift Correction", eq. cell_energy_clamp): the same result,
 * bit for bit, as dsmc_apply_pairs(kind, AUTO) followed by
 * dsmc_moment_match(mode, pair_cnt = pairs.cnt), with one read and one write
 * of each colliding cell's velocities.  cell_start[n_cells+1] as from
 * dsmc_sort_cells (every pair of cell k lies in [cell_start[k],
 * cell_start[k+1])); mom[6*n_cells] from dsmc_moment_match(CAPTURE) on the
 * pre-collision velocities; mode DSMC_MM_APPLY or DSMC_MM_APPLY_LITERAL.
 * Cells without pairs are left untouched; skipped cells (non-positive or
 * non-finite post value) count in st->mm_skipped (st may be NULL).
 * ws: the workspace the DEFER collide call filled (dsmc_collide_ws). */
int dsmc_apply_pairs_match(int32_t n_cells, const int32_t* cell_start, int32_t dtype,
                           dsmc_vec3 v, dsmc_pairs pairs, int32_t kind, const double* mom,
                           int32_t mode, void* ws, size_t ws_bytes, dsmc_status* st,
                           dsmc_stream_t stream);

/* Ab initio deflection angle by quadrature (section "Computational
 * Implementation: The Exact vs. Neural Paradigm"): for each of n pairs,
 * E = m_red g^2 / 2, r_min = largest root of 1 - b^2/r^2 - V(r)/E, and
 *   chi = pi - 2 b int_{r_min}^inf dr / (r^2 sqrt(1 - b^2/r^2 - V/E)),
 * evaluated after u = r_min / r and u = 1 - t^2 with Gauss-Legendre in t.
 * b (m), g (m/s) and chi (rad) are arrays of `dtype` (FP64 or FP32: the
 * arithmetic precision of the per-pair rule; for FP32 the root and
 * V(r_min) are finished in FP64 below the orbiting energy).  Pairs whose
 * integrand has a sharp peak near orbiting, or whose root is uncertain, are
 * re-evaluated in FP64 by a second pass (see dsmc_quad.refine); chi of such
 * a pair is written twice.  fold = 1 returns theta = arccos(cos chi) in
 * [0, pi].  A failed root search gives NaN and counts in st->root_fail. */
int dsmc_deflect_jager(int64_t n, int32_t dtype, const void* b, const void* g, void* chi,
                       double m_red, const dsmc_potential* pot, dsmc_quad quad, int32_t fold,
                       dsmc_status* st, dsmc_stream_t stream);

/* In-step ab initio rule: Phase A per accepted pair computes chi(b, g_pre)
 * by the quadrature above with b = b_max sqrt(1 - exp(-|z|^2/2)) from the
 * pair's latent z (b^2 uniform on [0, b_max^2]); Phase B rotates the current
 * v_r by chi about the azimuth direction of the latent xi. */
int dsmc_collide_jager(int32_t n_cells, int32_t dtype, dsmc_vec3 v, dsmc_pairs pairs,
                       dsmc_rng rng, double m_red, double b_max, const dsmc_potential* pot,
                       dsmc_quad quad, int32_t schedule, void* ws, size_t ws_bytes,
                       dsmc_status* st, dsmc_stream_t stream);

/* Neural collision operator (sections "Cell-Based Neural Collision
 * Operator" and "Hard Conservation via Projection and Pair Update"):
 * Phase A per accepted pair: x = [v_r/sigma_v, xi, z] -> y = f_theta(x) ->
 * u = y / max(|y|, 1e-30) (energy-shell projection; the isotropic direction
 * if |y| <= 1e-30); Phase B as in dsmc_collide_vhs.  Follow with
 * dsmc_moment_match(APPLY) for the paper's cell-wise correction.
 * ws: dsmc_collide_ws(cap, dtype) bytes for a BF16 network; the FP64/FP32
 * reference networks (wdtype == dtype) need dsmc_collide_ws(cap, dtype) +
 * dsmc_neural_act_bytes(net, cap). */
int dsmc_neural_collide(const dsmc_mlp* net, int32_t n_cells, int32_t dtype, dsmc_vec3 v,
                        dsmc_pairs pairs, dsmc_rng rng, int32_t schedule, void* ws,
                        size_t ws_bytes, dsmc_status* st, dsmc_stream_t stream);

/* Rows form of the surrogate for training: for B rows x[B][dims[0]] and
 * speeds g[B]: y_raw = f_theta(x) [B][dims[L]], vr_out = g * y/|y| [B][3].
 * Array dtype: FP32 for the BF16 network, FP64 for the FP64 network.
 * act_save (nullable): activations kept for dsmc_neural_backward, size
 * dsmc_neural_act_bytes(net, B); its contents are private to the pair of
 * calls (for the BF16 network: FP32 pre-activations and bf16 activations and
 * inputs, transposed in blocks of 128 rows). */
size_t dsmc_neural_act_bytes(const dsmc_mlp* net, int64_t B);
int dsmc_neural_forward_rows(const dsmc_mlp* net, int64_t B, const void* x, const void* g,
                             void* y_raw, void* vr_out, void* act_save, size_t act_bytes,
                             dsmc_stream_t stream);

/* Backward of the rows form (section "Neural Surrogate Training": the
 * surrogate is trained by gradient descent on its loss; this is the
 * hand-written adjoint of eq. mlp_output and of eq. energy_shell_projection):
 * given dL/dv_r' [B][3], writes dW[l], db[l]
 * (FP32 for the BF16 network, FP64 for the FP64 network; accumulate = 1 adds
 * to them) and, if dx != NULL, dL/dx [B][dims[0]].  The row reductions of dW
 * and db run in a fixed order (deterministic).  act_save from the forward
 * call with the same net and B; for the BF16 network x is not read again
 * (the forward saved it).
 * ws: dsmc_neural_backward_ws(net, B) bytes. */
size_t dsmc_neural_backward_ws(const dsmc_mlp* net, int64_t B);
int dsmc_neural_backward(const dsmc_mlp* net, int64_t B, const void* x, const void* act_save,
                         const void* y_raw, const void* g, const void* dL_dvr,
                         void* const* dW, void* const* db, void* dx, int32_t accumulate,
                         void* ws, size_t ws_bytes, dsmc_stream_t stream);

/* Adjoint of the centred moment matching of one cell group (eq.
 * cell_energy_clamp, section "Optional Cell-Wise Energy Drift Correction", in
 * the centred reading v -> u_pre + alpha (v - u_post)) with respect to the
 * post-collision velocities, for training through the matching:
 *   dL/dv_m = alpha (G_m - mean G) - (alpha / S_post) (sum_i G_i . c_i) c_m,
 * c = v - u_post.  FP64 arrays [3][n] SoA in sorted order, pre-moments from
 * CAPTURE.  Cells with N < 2 or S_post <= 0 pass G through. */
int dsmc_moment_match_backward(int32_t n_cells, const int32_t* cell_start, const double* mom_pre,
                               const double* v_post_x, const double* v_post_y,
                               const double* v_post_z, const double* G_x, const double* G_y,
                               const double* G_z, double* out_x, double* out_y,
                               double* out_z, dsmc_stream_t stream);

/* Training helpers.  MSE on the post-collision velocities of the pair,
 * L = (1/B) sum |v_r' - v_r'*|^2 / (4 sigma_v^2); writes dL/dv_r' and adds L
 * to *loss (device double; workgroup partial sums are added atomically, so
 * the last bits of L may differ between runs, dL/dv_r' does not).  Arrays
 * FP32 [B][3]. */
int dsmc_mse_loss(int64_t B, const float* vr_new, const float* vr_target, double sigma_v,
                  float* dL_dvr, double* loss, dsmc_stream_t stream);

/* MSE on the scattering directions (section "Neural Surrogate Training":
 * the surrogate's loss on the scattering directions): with g = |v_r'*|,
 * L = (1/B) sum |v_r' - v_r'*|^2 / (4 g^2) = (1/B) sum |u - u*|^2 / 4, the
 * velocity MSE above with each pair normalised by its own g^2; writes dL/dv_r'
 * and adds L to *loss (atomically per workgroup, as above).  Rows with
 * v_r'* = 0 contribute nothing.  Arrays FP32 [B][3]. */
int dsmc_direction_loss(int64_t B, const float* vr_new, const float* vr_target, float* dL_dvr,
                        double* loss, dsmc_stream_t stream);

/* Cosine learning-rate schedule of the surrogate training (section "Neural
 * Surrogate Training": Adam with a cosine schedule): the rate at step t of T,
 * lr_min + (lr_max - lr_min) (1 + cos(pi min(t, T) / T)) / 2, so lr_max at
 * t = 0 and lr_min from t = T on.  Host function; T < 1 returns lr_max. */
double dsmc_cosine_lr(int64_t t, int64_t T, double lr_max, double lr_min);

/* Adam (Kingma & Ba 2015) with bias correction on FP32 master parameters;
 * also writes the bf16 copy used by the MFMA forward when param_bf16 != NULL.
 * lr: the step's rate, e.g. dsmc_cosine_lr(t, T, lr_max, lr_min). */
int dsmc_adam_step(int64_t n, float* param, void* param_bf16, const float* grad, float* m,
                   float* v, int64_t t, double lr, double beta1, double beta2, double eps,
                   dsmc_stream_t stream);

/* Training rows from the quadrature ("physics harvesting" on pairs the
 * library generates): for rows (v_r, xi, z) in FP64, b from z as in
 * dsmc_collide_jager, chi by quadrature, target v_r' = g (cos chi vhat +
 * sin chi e_perp(xi)).  Also writes x = [v_r/sigma_v, xi, z] (FP32) and chi. */
int dsmc_harvest_rows(int64_t B, const double* vr, const double* xi, const double* z,
                      double sigma_v, double b_max, double m_red, const dsmc_potential* pot,
                      dsmc_quad quad, float* x_out, float* g_out, float* target_out,
                      double* chi_out, dsmc_status* st, dsmc_stream_t stream);

/* One persistent launch per step for the isotropic rule: workgroups take
 * cells from a work queue and, with the cell staged in LDS, run moments, NTC
 * selection, Phase A, Phase B and (match != 0) centred moment matching; HBM
 * sees one read and one write of the velocities.  Cells of up to 320
 * particles are taken by one-wave workgroups (many resident per CU); larger
 * ones are listed and taken by a second launch of block-wide workgroups.
 * Results are bit-identical to dsmc_moment_match(CAPTURE) ->
 * dsmc_select_pairs_ntc -> dsmc_collide_vhs -> dsmc_moment_match(APPLY) with
 * the same rng.  pair_cnt[n_cells] receives each cell's accepted pairs.
 * Accepted pairs beyond one LDS batch (256 in the wave form, 2048 in the
 * block form) are applied batch by batch in candidate order (same result); a
 * cell of more than 3072 particles (beyond the LDS staging) is left
 * unchanged with pair_cnt = -1 and DSMC_ST_PAIR_OVERFLOW set, for the
 * separate entry points to handle.
 * ws: dsmc_step_vhs_ws(n_cells, 0) bytes (queues and the list of large
 * cells). */
size_t dsmc_step_vhs_ws(int32_t n_cells, int64_t cap);
int dsmc_step_vhs_fused(int32_t n_cells, const int32_t* cell_start, int32_t dtype, dsmc_vec3 v,
                        dsmc_xs xs, const double* lambda, dsmc_rng rng, int32_t match,
                        int32_t* pair_cnt, void* ws, size_t ws_bytes, dsmc_status* st,
                        dsmc_stream_t stream);

/* Tuning knobs (host): threshold in pairs above which AUTO leaves the LANE
 * schedule; the autotuner in the Python package sets it. */
int dsmc_set_block_threshold(int32_t pairs);
int32_t dsmc_get_block_threshold(void);

/* Launch shape of dsmc_apply_pairs_match (process-wide, as the threshold
 * above): workgroups per compute unit of its three persistent kernels --
 * the wave-per-cell kernel, and the medium (256 lanes) and big (512 lanes)
 * block-per-cell kernels.  Every shape gives the same results bit for bit;
 * paper_2602_21244_amd/autotune.py measures them on the step's own pair
 * list and installs the fastest.  Defaults 40 / 2 / 1. */
typedef struct {
    int32_t wave_per_cu;    /* 1..256 */
    int32_t medium_per_cu;  /* 1..64 */
    int32_t big_per_cu;     /* 1..64 */
    int32_t reserved;
} dsmc_match_schedule;
int dsmc_set_match_schedule(const dsmc_match_schedule* ms);
int dsmc_get_match_schedule(dsmc_match_schedule* ms);

/* Chapman-Enskog viscosity from the deflection angle (section "Macroscopic
 * Validation: Viscosity and Transport Coefficients", eq. chapman_enskog):
 *   Q2(E) = 2 pi int_0^b_cut (1 - cos^2 chi(b, E)) b db   [m^2]
 * by composite Gauss-Legendre in b (n_panels equal panels of n_gl nodes, chi
 * by the quadrature of dsmc_deflect_jager in FP64); E in K (E_r / k_B),
 * b_cut in m.  ws: dsmc_transport_q2_ws bytes.  Root failures count in st. */
size_t dsmc_transport_q2_ws(int64_t n_E, int32_t n_panels, int32_t n_gl);
int dsmc_transport_q2(int64_t n_E, const double* E_kelvin, double b_cut, int32_t n_panels,
                      int32_t n_gl, const dsmc_potential* pot, dsmc_quad quad, double* Q,
                      void* ws, size_t ws_bytes, dsmc_status* st, dsmc_stream_t stream);
/* Omega(T) and mu(T) = 5/16 sqrt(pi m k_B T) / Omega for n_T temperatures
 * (device arrays, K; m the atomic mass in kg).  DSMC_CE_STANDARD:
 * Omega = 1/(4 (kT)^4) int E^3 Q2 exp(-E/kT) dE, the Chapman-Cowling average
 * (reading of the printed average; it gives the hard-sphere viscosity);
 * DSMC_CE_AS_PRINTED: Omega = 1/(2 (kT)^3) int E^2 Q2 exp(-E/kT) dE.  The
 * Maxwellian average by n_lag-point generalised Gauss-Laguerre in E/kT.
 * ws: dsmc_viscosity_ce_ws bytes. */
enum { DSMC_CE_STANDARD = 0, DSMC_CE_AS_PRINTED = 1 };
size_t dsmc_viscosity_ce_ws(int32_t n_T, int32_t n_panels, int32_t n_gl, int32_t n_lag);
int dsmc_viscosity_ce(int32_t n_T, const double* T, double m, double b_cut, int32_t n_panels,
                      int32_t n_gl, int32_t n_lag, int32_t mode, const dsmc_potential* pot,
                      dsmc_quad quad, double* omega, double* mu, void* ws, size_t ws_bytes,
                      dsmc_status* st, dsmc_stream_t stream);

/* ---------------------------------------------------------------------- */
/* Neural deflection-angle table (sections "Neural Network Architecture",
 * "Neural Surrogate Training" and "Runtime Acceleration via Neural Table
 * Look-up"): an angle network maps x = [2 (ln E - lne_lo)/(lne_hi - lne_lo)
 * - 1, b / b_max] (E = E_r / k_B in K) through SiLU hidden layers and a
 * Softplus output to a prediction y of ln(1 + theta), theta the folded
 * deflection angle arccos(cos chi) in [0, pi].  The network synthesises an
 * n_e x n_b table of theta on the grid ln E_i = lne_lo + i (lne_hi -
 * lne_lo)/(n_e - 1), b_j / b_max = j / (n_b - 1); a collision rule looks
 * theta up by bilinear interpolation (coordinates clamped to the grid). */
enum { DSMC_ANET_MAX_LAYERS = 8 };
typedef struct {
    int32_t n_layers;                       /* weight layers, 2..8 */
    int32_t dims[DSMC_ANET_MAX_LAYERS + 1]; /* dims[0] = 2, dims[n_layers] = 1, each <= 1024 */
    const void* W[DSMC_ANET_MAX_LAYERS];    /* bf16 [dims[l+1]][dims[l]] row-major (device) */
    const float* b[DSMC_ANET_MAX_LAYERS];   /* fp32 [dims[l+1]] (device) */
} dsmc_anet;

typedef struct {
    int32_t n_e, n_b;        /* grid nodes along ln E and b / b_max, each >= 2 */
    double lne_lo, lne_hi;   /* ln(E / K) range of the grid, lne_lo < lne_hi */
    float* theta;            /* [n_e][n_b] folded angle in rad (device) */
} dsmc_chi_table;

/* Workspace for dsmc_anet_forward / dsmc_anet_backward on `rows` rows
 * (activations of every layer are kept for the backward). */
size_t dsmc_anet_ws(const dsmc_anet* net, int64_t rows);
/* y[rows] = network(x[rows][2]) (BF16 matrix cores, FP32 accumulation).
 * The activations stay in ws for a following dsmc_anet_backward. */
int dsmc_anet_forward(const dsmc_anet* net, int64_t rows, const float* x, float* y, void* ws,
                      size_t ws_bytes, dsmc_stream_t stream);
/* Gradients of sum_r dy[r] y[r] for the rows of the preceding forward on the
 * same ws: dW[l] fp32 [dims[l+1]][dims[l]], db[l] fp32 [dims[l+1]]
 * (overwritten; reductions in a fixed order). */
int dsmc_anet_backward(const dsmc_anet* net, int64_t rows, const float* dy, float* const* dW,
                       float* const* db, void* ws, size_t ws_bytes, dsmc_stream_t stream);
/* Mean Huber loss (threshold 1) of yhat against y (eq. huber_loss) into
 * *loss (FP64, device) and its gradient dy = clip(yhat - y, -1, 1) / n. */
int dsmc_huber_loss(int64_t n, const float* yhat, const float* y, float* dy, double* loss,
                    dsmc_stream_t stream);
/* Training rows from quadrature results (b in m, g in m/s, chi in rad, FP64):
 * x[n][2] as above with E = m_red g^2 / (2 k_B), y[n] = ln(1 + theta). */
int dsmc_anet_rows(int64_t n, const double* b, const double* g, const double* chi,
                   double m_red, double lne_lo, double lne_hi, double b_max, float* x,
                   float* y, dsmc_stream_t stream);
/* Synthesise tab->theta from the network: theta = clip(exp(y) - 1, 0, pi).
 * ws: dsmc_chi_table_ws bytes. */
size_t dsmc_chi_table_ws(const dsmc_anet* net, const dsmc_chi_table* tab);
int dsmc_chi_table_build(const dsmc_anet* net, const dsmc_chi_table* tab, void* ws,
                         size_t ws_bytes, dsmc_stream_t stream);
/* Table rule: Phase A per accepted pair looks theta up at E = m_red g_pre^2 /
 * (2 k_B) and b / b_max = sqrt(U4) (the latent impact parameter of
 * dsmc_collide_jager); Phase B rotates the current v_r by theta about the
 * azimuth direction of xi.  ws: dsmc_collide_ws(cap, dtype) bytes. */
int dsmc_collide_table(const dsmc_chi_table* tab, int32_t n_cells, int32_t dtype, dsmc_vec3 v,
                       dsmc_pairs pairs, dsmc_rng rng, double m_red, int32_t schedule, void* ws,
                       size_t ws_bytes, dsmc_stream_t stream);

/* ---------------------------------------------------------------------- */
/* The flow loop around the collision step (section "Results and
 * Discussion": the Couette channel and the lid-driven cavity).  The paper
 * gives no formulas for it; the standard DSMC method is used (Bird 1994).  */

/* Box of nx x ny uniform cells over [0, Lx] x [0, Ly] (unit depth in z).
 * Sides 0..3 are x = 0, x = Lx, y = 0, y = Ly, each periodic (the opposite
 * side must be periodic too), specular, or diffuse with wall temperature
 * T_w[side] (K) and wall velocity u_w[side] (m/s; its tangential components
 * are used).  m: particle mass (kg).  Passed by host pointer, read at call. */
enum { DSMC_WALL_PERIODIC = 0, DSMC_WALL_SPECULAR = 1, DSMC_WALL_DIFFUSE = 2 };
typedef struct {
    int32_t nx, ny;
    double Lx, Ly;
    int32_t kind[4];
    double T_w[4];
    double u_w[4][3];
    double m;
} dsmc_domain;

/* Move step: every particle flies dt ballistically; when it reaches a side
 * first, the remaining time continues after the side's rule: periodic shifts
 * by the period, specular flips the normal velocity, diffuse re-emits from
 * the wall Maxwellian (normal speed sigma_w sqrt(-2 ln(1 - U1)), tangential
 * u_w + sigma_w n, n a Box-Muller pair of (U2, U3), sigma_w = sqrt(k T_w/m)),
 * with U1, U2 from Philox(slot s, event h, step, 6) and U3 from (.., 7), s
 * the particle's index in the arrays.  At most 8 wall events per particle and
 * call (more: the flight is finished without further events, counted in
 * st->wall_limit with DSMC_ST_WALL_LIMIT); st->wall_events counts events.
 * Positions are clamped to the box, then cell_of[s] = iy nx + ix with
 * ix = floor(x nx / Lx) (of the stored position), clamped to the grid.
 * pos.x, pos.y: positions (pos.z unused); v: velocities; both in place, of
 * `dtype`; arithmetic in FP64.  st may be NULL. */
int dsmc_move(int32_t n, int32_t dtype, dsmc_vec3 pos, dsmc_vec3 v, const dsmc_domain* dom,
              double dt, dsmc_rng rng, int32_t* cell_of, dsmc_status* st,
              dsmc_stream_t stream);

/* out.c[s] = in.c[perm[s]] for each component c whose pointers are both
 * non-NULL (the positions into the cell order of dsmc_sort_cells). */
int dsmc_gather(int32_t n, int32_t dtype, const int32_t* perm, dsmc_vec3 in, dsmc_vec3 out,
                dsmc_stream_t stream);

/* Sampling of the macroscopic fields: per cell k, acc[13k .. 13k+12] +=
 * (N, sum v_x, v_y, v_z, sum v_x^2, v_y^2, v_z^2, v_x v_y, v_x v_z, v_y v_z,
 * sum |v|^2 v_x, |v|^2 v_y, |v|^2 v_z) over the cell's sorted slots, FP64. */
int dsmc_sample(int32_t n_cells, const int32_t* cell_start, int32_t dtype, dsmc_vec3 v,
                double* acc, dsmc_stream_t stream);

/* Fields from n_samples accumulated samples: fields[9k ..] = (number
 * density, u_x, u_y, u_z, T = m <|c|^2> / (3 k), tau_xy = -rho <c_x c_y>,
 * q_x, q_y, q_z with q = rho <|c|^2 c> / 2), c = v - u, rho = n m, number
 * density = N / n_samples * fnum_per_volume (F_N / V_cell).  Cells never
 * sampled give zeros. */
int dsmc_sample_fields(int32_t n_cells, const double* acc, double n_samples, double mass,
                       double fnum_per_volume, double* fields, dsmc_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* DSMC_H */
