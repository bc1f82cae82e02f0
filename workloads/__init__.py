"""Seeded synthetic inputs for the DSMC collision step.

This module is shared by the CPU oracle and the GPU path, so it holds input
data and input recipes only: particle populations, cell ids, velocities, pair
batches, physical parameter sets and network initialisations.  It contains
none of the collision method's arithmetic (no cross sections applied to pairs,
no selection, scattering, quadrature or moment matching).

Every generator is driven by ``numpy.random.default_rng(seed)``.  The shapes,
densities and temperatures follow the workloads described in the paper's
results sections (relaxation, lid-driven cavity, Mach-10 cylinder, the
physics-harvesting dataset); none of the paper's own data exists here, so these
synthetic populations stand in for it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# Physical constants and parameter sets (data, not method arithmetic)
# --------------------------------------------------------------------------
KB = 1.380649e-23          # Boltzmann constant, J/K (exact SI value)
AMU = 1.66053906660e-27    # atomic mass unit, kg

# Argon VHS parameters (the values quoted for the paper's argon cases; VHS law
# itself is Bird's).
AR_MASS = 6.63e-26         # kg
AR_D_REF = 4.17e-10        # m
AR_OMEGA = 0.81
AR_T_REF = 273.0           # K

# Collision probability per particle per step used to fix the collision-rate
# parameter lambda = F_N * dt / V_c (the paper gives no time step).
P_COLL = 0.5

# Impact-parameter cut-off for the ab initio path (m).
B_MAX = 1.0e-9


@dataclass(frozen=True)
class JagerParams:
    """Coefficients of the modified Tang-Toennies Ar-Ar potential form.

    Units: r in Angstrom, V/k_B in Kelvin.  The functional form is the paper's
    (Born-Mayer exponential minus damped C6..C16 dispersion for r >= 0.4 R_eps,
    screened Coulomb below).  The paper does not print the coefficient values.

    PLACEHOLDER SET: the dispersion coefficients and the shape exponents
    a2, a_-1, a_-2, beta_tt are typical Ar2 magnitudes; A and a1 were fitted so
    the well sits at R_eps = 3.757 A with depth 143.2 K (the known Ar2 well), and
    the short-range pair (A_sr, a_sr) was fitted for continuity of V and V' at
    0.4 R_eps.  It is NOT the published Jager et al. (2009) set.  Every entry
    point takes the coefficients as input, so the published set can be passed
    in unchanged when available.
    """
    A: float = 42794676.32833092          # K
    a1: float = -2.9242605940585715       # 1/A
    a2: float = -9.71208881e-2            # 1/A^2
    am1: float = 2.75206827e-2            # A
    am2: float = -1.01489050              # A^2
    beta_tt: float = 4.02517211           # 1/A  (Tang-Toennies damping constant)
    C: tuple = (4.42812017e5, 3.26707684e6, 2.45656537e7,
                2.21602374e8, 2.52700144e9, 3.52802239e10)  # C6..C16, K*A^(2n)
    R_eps: float = 3.757                  # A
    A_sr: float = 4736176.6454498805      # K*A
    a_sr: float = 1.8929614359536953      # 1/A


JAGER_PLACEHOLDER = JagerParams()


def maxwell_sigma(T: float, m: float = AR_MASS) -> float:
    """Standard deviation of one Maxwellian velocity component (m/s)."""
    return math.sqrt(KB * T / m)


def vhs_mean_sigma_g(T: float, m=AR_MASS, d_ref=AR_D_REF, omega=AR_OMEGA,
                     T_ref=AR_T_REF) -> float:
    """Maxwellian average <sigma_T g> of the VHS law (closed form, Bird 1994).

    Used only to choose the collision-rate parameter of a workload.
    """
    return 4.0 * d_ref ** 2 * math.sqrt(math.pi * KB * T_ref / m) * (T / T_ref) ** (1.0 - omega)


def hs_mean_sigma_g(T: float, sigma: float, m=AR_MASS) -> float:
    """<sigma g> for a constant cross section: sigma * mean relative speed."""
    return sigma * math.sqrt(16.0 * KB * T / (math.pi * m))


# --------------------------------------------------------------------------
# Particle populations
# --------------------------------------------------------------------------
@dataclass
class Population:
    """Particles in original (unsorted) order plus per-cell parameters."""
    n_cells: int
    cell_of: np.ndarray          # int32 [N]
    v: np.ndarray                # float64 [3, N]  (SoA)
    lam: np.ndarray              # float64 [n_cells], lambda_k = F_N dt / V_c
    xs: dict                     # cross-section description
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.cell_of.shape[0])


def _vhs_xs():
    return {"kind": "vhs", "m": AR_MASS, "d_ref": AR_D_REF, "omega": AR_OMEGA,
            "T_ref": AR_T_REF}


def vhs_argon_1d(seed: int = 1, n: int = 20000, n_cells: int = 200,
                 T: float = 273.0, shear: float = 50.0) -> Population:
    """Relaxation-style VHS argon population in 1D cells.

    Cell id uniform in [0, n_cells) (counts ~ Poisson(n/n_cells)), shuffled
    order, Maxwellian at T plus a linear shear u_x = -shear..+shear across the
    cells.  lambda gives P_COLL accepted pairs per particle per step on average.
    """
    rng = np.random.default_rng(seed)
    cell_of = rng.integers(0, n_cells, size=n, dtype=np.int64).astype(np.int32)
    s = maxwell_sigma(T)
    v = rng.normal(0.0, s, size=(3, n))
    ux = -shear + 2.0 * shear * (cell_of.astype(np.float64) + 0.5) / n_cells
    v[0] += ux
    nbar = n / n_cells
    lam_val = 2.0 * P_COLL / (max(nbar - 1.0, 1.0) * vhs_mean_sigma_g(T))
    lam = np.full(n_cells, lam_val)
    return Population(n_cells, cell_of, v, lam, _vhs_xs(), name="vhs_argon_1d",
                      meta={"T": T, "seed": seed})


def cavity_grid(seed: int = 3, nx: int = 200, ny: int = 200, mean: float = 25.0,
                lid_factor: float = 4.0, T: float = 273.15, u_lid: float = 100.0,
                shuffle: bool = True) -> Population:
    """Cavity-like 2D grid: Poisson(mean) per cell, lid row at lid_factor*mean.

    Velocities: Maxwellian at T plus u_x = u_lid * row/(ny-1) (row ny-1 is the
    lid).  Uniform lambda chosen for P_COLL at the bulk density.
    """
    rng = np.random.default_rng(seed)
    n_cells = nx * ny
    means = np.full(n_cells, mean)
    means[(ny - 1) * nx:] = mean * lid_factor
    counts = rng.poisson(means).astype(np.int64)
    cell_of = np.repeat(np.arange(n_cells, dtype=np.int32), counts)
    n = cell_of.shape[0]
    row = (cell_of // nx).astype(np.float64)
    v = rng.normal(0.0, maxwell_sigma(T), size=(3, n))
    v[0] += u_lid * row / (ny - 1)
    if shuffle:
        p = rng.permutation(n)
        cell_of = cell_of[p]
        v = v[:, p]
    lam_val = 2.0 * P_COLL / ((mean - 1.0) * vhs_mean_sigma_g(T))
    lam = np.full(n_cells, lam_val)
    return Population(n_cells, np.ascontiguousarray(cell_of), np.ascontiguousarray(v),
                      lam, _vhs_xs(), name="cavity_grid",
                      meta={"nx": nx, "ny": ny, "seed": seed})


def cylinder_grid(seed: int = 5, nx: int = 400, ny: int = 300, cx: float = 150.0,
                  cy: float = 150.0, radius: float = 40.0, band: float = 55.0,
                  n_free: float = 222.0, band_factor: float = 10.0,
                  T_free: float = 200.0, u_free: float = 2630.0,
                  T_band: float = 6400.0, u_band: float = 263.0,
                  order: str = "realistic", move_frac: float = 0.3,
                  scale: float = 1.0) -> Population:
    """Mach-10 cylinder-shaped step population.

    Empty disc of `radius` cells around (cx, cy); an upstream half-annulus
    radius < r <= band holds band_factor x the free-stream density at the
    post-shock temperature and bulk velocity; all other cells hold the
    free-stream (T_free, u_free).  Constant cross section pi*B_MAX^2 with a
    per-cell lambda for P_COLL at each region's expected density.

    order: "sorted" (cell-sorted), "realistic" (cell-sorted, then move_frac of
    particles get their cell id moved by +-1 in x, as after a streaming step),
    or "shuffled" (random order).  `scale` multiplies the densities (used for
    reduced-size parity cases).
    """
    rng = np.random.default_rng(seed)
    n_cells = nx * ny
    ix = np.arange(n_cells) % nx
    iy = np.arange(n_cells) // nx
    dx = ix + 0.5 - cx
    dy = iy + 0.5 - cy
    r = np.sqrt(dx * dx + dy * dy)
    inside = r <= radius
    in_band = (~inside) & (r <= band) & (dx < 0.0)
    dens = np.where(inside, 0.0, np.where(in_band, n_free * band_factor, n_free)) * scale
    counts = rng.poisson(dens).astype(np.int64)
    cell_of = np.repeat(np.arange(n_cells, dtype=np.int32), counts)
    n = cell_of.shape[0]
    is_band = np.repeat(in_band, counts)
    T = np.where(is_band, T_band, T_free)
    s = np.sqrt(KB * T / AR_MASS)
    v = rng.standard_normal(size=(3, n)) * s
    v[0] += np.where(is_band, u_band, u_free)
    if order == "realistic":
        mv = rng.random(n) < move_frac
        step = np.where(rng.random(n) < 0.5, -1, 1)
        cx_new = np.clip(cell_of % nx + step, 0, nx - 1)
        moved = (cell_of // nx) * nx + cx_new
        cell_of = np.where(mv, moved, cell_of).astype(np.int32)
    elif order == "shuffled":
        p = rng.permutation(n)
        cell_of = cell_of[p]
        v = v[:, p]
    elif order != "sorted":
        raise ValueError(order)
    sigma = math.pi * B_MAX ** 2
    lam = np.zeros(n_cells)
    free = (~inside) & (~in_band)
    nf, nb = n_free * scale, n_free * band_factor * scale
    if nf > 1.0:
        lam[free] = 2.0 * P_COLL / ((nf - 1.0) * hs_mean_sigma_g(T_free, sigma))
    if nb > 1.0:
        lam[in_band] = 2.0 * P_COLL / ((nb - 1.0) * hs_mean_sigma_g(T_band, sigma))
    xs = {"kind": "const", "sigma": sigma, "m": AR_MASS}
    return Population(n_cells, np.ascontiguousarray(cell_of, dtype=np.int32),
                      np.ascontiguousarray(v), lam, xs, name="cylinder_grid",
                      meta={"nx": nx, "ny": ny, "seed": seed, "order": order})


def ragged_population(seed: int, n_cells: int, max_count: int, T: float = 300.0,
                      xs: str = "vhs", empty_frac: float = 0.2,
                      lam_scale: float = 1.0) -> Population:
    """Small irregular population for parity edge cases.

    Cell counts are drawn uniformly in [0, max_count] with a fraction of empty
    and single-particle cells, in shuffled order.
    """
    rng = np.random.default_rng(seed)
    counts = rng.integers(0, max_count + 1, size=n_cells)
    counts[rng.random(n_cells) < empty_frac] = 0
    counts[rng.random(n_cells) < 0.05] = 1
    cell_of = np.repeat(np.arange(n_cells, dtype=np.int32), counts)
    n = cell_of.shape[0]
    v = rng.normal(0.0, maxwell_sigma(T), size=(3, n))
    v[0] += rng.normal(0, 50.0, size=n_cells)[cell_of] if n else 0.0
    p = rng.permutation(n)
    cell_of = cell_of[p]
    v = v[:, p]
    nbar = max(float(counts.mean()), 2.0)
    if xs == "vhs":
        x = _vhs_xs()
        lam_val = 2.0 * P_COLL / ((nbar - 1.0) * vhs_mean_sigma_g(T))
    else:
        sigma = math.pi * B_MAX ** 2
        x = {"kind": "const", "sigma": sigma, "m": AR_MASS}
        lam_val = 2.0 * P_COLL / ((nbar - 1.0) * hs_mean_sigma_g(T, sigma))
    lam = np.full(n_cells, lam_val * lam_scale) * rng.uniform(0.5, 1.5, size=n_cells)
    return Population(n_cells, np.ascontiguousarray(cell_of), np.ascontiguousarray(v),
                      lam, x, name="ragged", meta={"seed": seed})


# --------------------------------------------------------------------------
# Ab initio deflection batches and training rows
# --------------------------------------------------------------------------
def deflection_batch(seed: int = 2, n: int = 1 << 20, g_lo: float = 100.0,
                     g_hi: float = 20000.0, b_max: float = B_MAX):
    """(b, g) pairs: g log-uniform on [g_lo, g_hi], b^2 uniform on [0, b_max^2].

    Returns b (m), g (m/s) as float64 arrays and the reduced mass (kg).
    """
    rng = np.random.default_rng(seed)
    g = g_lo * (g_hi / g_lo) ** rng.random(n)
    b = b_max * np.sqrt(rng.random(n))
    return b, g, AR_MASS / 2.0


def training_rows(seed: int = 4, n: int = 65536, g_lo: float = 100.0,
                  g_hi: float = 20000.0):
    """Harvested-pair rows for surrogate training.

    v_r: isotropic direction times g (log-uniform on [g_lo, g_hi]);
    xi (3) and z (2): independent N(0,1) latents.  The impact parameter of a
    row is the one its z encodes (b^2/b_max^2 = 1 - exp(-|z|^2/2), which is
    uniform).  sigma_v = sqrt(<|v_r|^2>/3) over the rows.
    """
    rng = np.random.default_rng(seed)
    g = g_lo * (g_hi / g_lo) ** rng.random(n)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    vr = d * g[:, None]
    xi = rng.standard_normal((n, 3))
    z = rng.standard_normal((n, 2))
    sigma_v = float(np.sqrt(np.mean(g * g) / 3.0))
    return {"vr": vr, "xi": xi, "z": z, "g": g, "sigma_v": sigma_v}


def angle_samples(seed: int = 11, n: int = 1 << 20, lne_lo: float = math.log(5.0),
                  lne_hi: float = math.log(5.0e5), m_red: float = AR_MASS / 2,
                  b_max: float = B_MAX):
    """Collision parameters for the angle network's training set.

    E_r / k_B log-uniform on [exp(lne_lo), exp(lne_hi)] K; b / b_max uniform
    for one half of the rows and U^2 (biased towards head-on collisions) for
    the other half; g = sqrt(2 E_r / m_red).
    """
    rng = np.random.default_rng(seed)
    lnE = rng.uniform(lne_lo, lne_hi, n)
    E = np.exp(lnE) * KB
    u = rng.random(n)
    b_rel = np.where(np.arange(n) % 2 == 0, u, u * u)
    g = np.sqrt(2.0 * E / m_red)
    return {"b": b_rel * b_max, "g": g, "E_kelvin": np.exp(lnE), "b_rel": b_rel}


# --------------------------------------------------------------------------
# Network parameters
# --------------------------------------------------------------------------
def mlp_init(seed: int, dims, scale: float = 1.0):
    """PyTorch-default-style uniform init: W, b ~ U(-1/sqrt(fan_in), +)."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for l in range(len(dims) - 1):
        k = 1.0 / math.sqrt(dims[l])
        Ws.append(rng.uniform(-k, k, size=(dims[l + 1], dims[l])) * scale)
        bs.append(rng.uniform(-k, k, size=(dims[l + 1],)) * scale)
    return Ws, bs


SURROGATE_DIMS = (8, 128, 128, 128, 128, 3)
FD_DIMS = (8, 16, 3)


# --------------------------------------------------------------------------
# Flow cases around the collision step (section "Results and Discussion")
# --------------------------------------------------------------------------
WALL_PERIODIC, WALL_SPECULAR, WALL_DIFFUSE = 0, 1, 2


@dataclass
class Flow:
    """A gas in a box of nx x ny cells over [0, Lx] x [0, Ly] (unit depth in
    z): positions pos[2, N], velocities v[3, N], per-side wall description
    (x = 0, x = Lx, y = 0, y = Ly), time step and collision-rate parameter
    lam = F_N dt / V_c per cell."""
    nx: int
    ny: int
    Lx: float
    Ly: float
    kinds: tuple
    T_w: tuple
    u_w: tuple
    pos: np.ndarray
    v: np.ndarray
    dt: float
    lam: np.ndarray
    xs: dict
    n_density: float
    fnum_per_volume: float      # F_N / V_c
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.pos.shape[1])

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny


def _hs_mean_free_path_density(kn_length: float) -> float:
    """Number density whose hard-sphere mean free path 1/(sqrt(2) pi d^2 n),
    with the argon VHS reference diameter, equals kn_length (the reading of
    the paper's Knudsen numbers: Kn = lambda / L)."""
    return 1.0 / (math.sqrt(2.0) * math.pi * AR_D_REF ** 2 * kn_length)


def _fill(rng, n, Lx, Ly, T, u):
    pos = np.stack([rng.uniform(0.0, Lx, n), rng.uniform(0.0, Ly, n)])
    v = rng.normal(0.0, maxwell_sigma(T), size=(3, n))
    v[0] += u[0]
    v[1] += u[1]
    return pos, v


def _time_step(n_density, dx, u_max, T):
    """A fifth of the hard-sphere mean collision time, and no more than a
    third of a cell crossed at u_max + 3 most-probable speeds."""
    c_mean = math.sqrt(8.0 * KB * T / (math.pi * AR_MASS))
    lam_mfp = 1.0 / (math.sqrt(2.0) * math.pi * AR_D_REF ** 2 * n_density)
    c_mp = math.sqrt(2.0 * KB * T / AR_MASS)
    return min(0.2 * lam_mfp / c_mean, dx / (3.0 * (u_max + 3.0 * c_mp)))


def couette_flow(seed: int = 7, ny: int = 50, ppc: int = 100, L: float = 1.0e-3,
                 kn: float = 0.2, u_wall: float = 500.0, T_wall: float = 273.0) -> Flow:
    """Planar Couette flow of argon (the paper's rarefied Couette case): walls
    at y = 0 and y = L moving at -u_wall and +u_wall in x, diffuse at T_wall;
    periodic in x over one cell width; gas initially at rest at T_wall."""
    rng = np.random.default_rng(seed)
    n_cells = ny
    n = ppc * n_cells
    dy = L / ny
    Lx = dy
    pos, v = _fill(rng, n, Lx, L, T_wall, (0.0, 0.0))
    nd = _hs_mean_free_path_density(kn * L)
    dt = _time_step(nd, dy, u_wall, T_wall)
    lam = np.full(n_cells, nd * dt / ppc)
    return Flow(1, ny, Lx, L, (WALL_PERIODIC, WALL_PERIODIC, WALL_DIFFUSE, WALL_DIFFUSE),
                (T_wall,) * 4,
                ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (-u_wall, 0.0, 0.0), (u_wall, 0.0, 0.0)),
                pos, v, dt, lam, _vhs_xs(), nd, nd / ppc, name="couette")


def cavity_flow(seed: int = 8, nx: int = 50, ny: int = 50, ppc: int = 100,
                L: float = 1.0e-3, kn: float = 0.1, u_lid: float = 100.0,
                T_wall: float = 273.15) -> Flow:
    """Lid-driven cavity of argon (the paper's generalisation test: side L =
    1 mm, 50 x 50 cells, 100 particles per cell, Kn = 0.1, lid at y = L moving
    at u_lid in x, all walls diffuse at T_wall); gas initially at rest."""
    rng = np.random.default_rng(seed)
    n_cells = nx * ny
    n = ppc * n_cells
    pos, v = _fill(rng, n, L, L, T_wall, (0.0, 0.0))
    nd = _hs_mean_free_path_density(kn * L)
    dt = _time_step(nd, L / max(nx, ny), u_lid, T_wall)
    lam = np.full(n_cells, nd * dt / ppc)
    return Flow(nx, ny, L, L, (WALL_DIFFUSE,) * 4, (T_wall,) * 4,
                ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (u_lid, 0.0, 0.0)),
                pos, v, dt, lam, _vhs_xs(), nd, nd / ppc, name="cavity")
