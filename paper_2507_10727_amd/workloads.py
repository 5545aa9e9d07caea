"""Seeded synthetic workloads for the RZ PIC-MCC timestep.

This module only *generates inputs*: problem presets, the static magnetron
field, the electron-argon cross-section tables and the initial particle load.
It holds none of the timestep's arithmetic (no gather, push, collision,
deposit, field solve or circuit), so that the GPU library and the CPU oracle
can both consume exactly the same inputs without sharing any method code.

Physical setting (paper, Sections 3-4): a dc magnetron discharge in argon,
2D R-Z with azimuthal symmetry, cathode on the z = 0 plane, anode at
z = Z_max, a static magnetic field from magnets behind the cathode, electron
impact elastic / excitation / ionization collisions with a uniform neutral
background, ion-induced secondary emission at the cathode, and a cathode that
floats through an external resistor.  The sizes below are synthetic stand-ins
in the paper's regime (densities 1e15-1e17 m^-3, 1-30 mTorr, 300-700 V
cathode, Introduction); the paper's own VSim inputs (QDB cross sections, the
two-magnet scalar-potential field) are not available and are replaced by the
analytic forms documented here.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# CODATA 2018 values (SI).  Each consumer keeps its own copy; these are used
# here only to build inputs (weights, thermal speeds, gas density for the
# cross-section tables is *not* computed here).
E_CHARGE = 1.602176634e-19
M_E = 9.1093837015e-31
AMU = 1.66053906660e-27
M_AR = 39.948 * AMU
K_B = 1.380649e-23
MU0 = 4e-7 * math.pi
TORR = 133.322368  # Pa

MC_PIC = 0
EC_PIC = 1
F32 = 0
F64 = 1
FIXED_V = 0
RESISTOR = 1
ABSORB = 0
REFLECT = 1
POISSON_MGCG = 0       # field-solve preconditioner: multigrid
POISSON_LEARNED = 1    # learned network (flexible CG)
POISSON_CG = 2         # none
POISSON_DIRECT = 3     # direct sine-transform solve (cathode covering z = 0)


@dataclasses.dataclass
class Problem:
    """One discharge: geometry, numerics, circuit, gas and species.

    Grid sizes are numbers of *cells*; the node grid is (nr+1) x (nz+1), node
    (i, j) at r = i*dr, z = j*dz, stored at linear index j*(nr+1)+i.
    """

    name: str = "custom"
    nr: int = 64
    nz: int = 64
    lr: float = 0.02
    lz: float = 0.02
    dt: float = 5e-12
    scheme: int = MC_PIC
    precision: int = F64
    cathode_rmax: Optional[float] = None  # defaults to lr (whole z = 0 plane)
    circuit: int = FIXED_V
    v_fixed: float = -400.0
    v_ext: float = -400.0
    r_ext: float = 100.0
    gamma_i: float = 0.1
    gamma_e: float = 0.0        # electron-induced yield (Section 3: 0.1)
    n_meta: float = 0.0         # static Ar* density (Section 3: 2.5e17 m^-3)
    e_iz_meta: float = 4.20     # ionization threshold from Ar* (eV)
    deposit_fixed: int = 0      # 1: fixed-point node charge (FP64, bit-reproducible)
    p_gas: float = 5e-3 * TORR
    t_gas: float = 300.0
    e_exc: float = 11.5
    e_iz: float = 15.76
    b_peak: float = 0.03
    density: float = 1e15
    te_ev: float = 2.0
    ti_ev: float = 0.03
    n_per_species: int = 200_000
    steps: int = 200
    seed: int = 250710727
    run: int = 0
    sort_every: int = 20
    poisson_rtol: float = 1e-8
    poisson_maxit: int = 200
    wall_bc: tuple = (ABSORB, ABSORB, ABSORB)
    frozen_ions: int = 0
    mcc_on: int = 1
    see_on: int = 1
    field_solve: int = 1
    extra_current: float = 0.0
    capacity_factor: float = 1.5
    poisson_mode: int = 0       # 0 multigrid, 1 learned network, 2 none (plain CG), 3 direct
    pc_batch: int = 0           # training batch of the learned preconditioner
    pc_maxit: int = 0           # learned iterations before the multigrid fallback
    pc_pre: int = 1             # learned preconditioner's first step: 1 V-cycle, 0 GS pair
    weight: Optional[float] = None  # macroparticle weight; default n*V/N
    cluster: float = 0.0        # fraction of each species loaded in the ring
    #                             0.35 R < r < 0.5 R, z < 0.1 L (deposit stress)
    magnets: int = 0            # 0: one current loop; 1: the two-magnet layout

    def __post_init__(self):
        if self.cathode_rmax is None:
            self.cathode_rmax = self.lr

    @property
    def dr(self) -> float:
        return self.lr / self.nr

    @property
    def dz(self) -> float:
        return self.lz / self.nz

    @property
    def nodes(self) -> int:
        return (self.nr + 1) * (self.nz + 1)

    @property
    def volume(self) -> float:
        return math.pi * self.lr ** 2 * self.lz

    def macro_weight(self) -> float:
        if self.weight is not None:
            return self.weight
        return self.density * self.volume / max(self.n_per_species, 1)

    def species(self):
        """(q, m, w) for electrons (0) and Ar+ (1)."""
        w = self.macro_weight()
        return ((-E_CHARGE, M_E, w), (E_CHARGE, M_AR - M_E, w))

    def capacity(self):
        c = int(self.n_per_species * self.capacity_factor) + 4096
        return (c, c)

    def replace(self, **kw) -> "Problem":
        # a cathode spanning the whole z = 0 plane keeps doing so when lr changes
        if "lr" in kw and "cathode_rmax" not in kw and self.cathode_rmax == self.lr:
            kw["cathode_rmax"] = kw["lr"]
        return dataclasses.replace(self, **kw)


# ---------------------------------------------------------------------------
# Presets (synthetic stand-ins in the paper's regime)
# ---------------------------------------------------------------------------

def unknown_mask(p: Problem) -> np.ndarray:
    """True on the nodes the field solve determines: all but the anode row
    (j = nz), the outer column (i = nr) and the cathode nodes of z = 0
    (r < cathode_rmax).  Node-major (j * (nr + 1) + i)."""
    j, i = np.divmod(np.arange(p.nodes), p.nr + 1)
    dirichlet = (j == p.nz) | (i == p.nr) | ((j == 0) & (i * (p.lr / p.nr) < p.cathode_rmax))
    return ~dirichlet


def random_potentials(p: Problem, n: int, seed: int) -> list:
    """Random potentials: white noise smoothed by a Gaussian of 0.7 to 24
    cells (cycling through six scales), unit rms, zero on Dirichlet nodes."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    unk = unknown_mask(p)
    out = []
    for k in range(n):
        s = (0.7, 1.5, 3.0, 6.0, 12.0, 24.0)[k % 6]
        f = gaussian_filter(rng.normal(size=(p.nz + 1, p.nr + 1)), s).ravel()
        f = np.where(unk, f, 0.0)
        out.append(f / np.sqrt(np.mean(f[unk] ** 2)))
    return out


def preset(name: str) -> Problem:
    """Named workloads.

    small_mc64_f64   : 64x64 cells over 2x2 cm, 2e5 e- + 2e5 Ar+, n = 1e15,
                       MC-PIC, FP64 state, cathode fixed at -400 V, 5 mTorr,
                       peak B 0.03 T, 200 steps (the small parity case).
    All three solve the field with the direct sine-transform solve (their
    cathode covers the z = 0 row); replace(poisson_mode=...) selects the
    conjugate-gradient solves.
    ec256x512_f32    : 256x512 cells over 4x8 cm, 1e7 + 1e7, n = 1e16,
                       EC-PIC, FP32 state, -500 V through 100 ohm, 10 mTorr,
                       peak B 0.05 T (the throughput case; mc256x512_f32 is
                       the same with the MC gather).
    ec512x1024_f32   : 512x1024 cells over 5x10 cm, 5e7 + 5e7, n = 1e17,
                       20 mTorr, -500 V through 10/100 ohm (high-density case;
                       mc512x1024_f32 the same with the MC gather).
    magnetron3x3_ec_f32 : the geometry of Section 3: 3 x 3 cm, 128 x 128
                       cells, cathode over 0.85 L_r and a Neumann block
                       beyond, the two-magnet field, -300 V through 3000 ohm,
                       ion yield 0.1, electron yield 0.1, Ar* 2.5e17 m^-3,
                       10 mTorr, EC-PIC (mc: MC-PIC), multigrid field solve,
                       seeded with 2e5 + 2e5 at 1e15 m^-3 (capacity 20x for
                       the discharge to grow).
    ec512x1024_clustered_f32 : the high-density case with half of each
                       species in the ring 0.35 R < r < 0.5 R, z < 0.1 L (the
                       magnetised ring above the cathode): about 3e3
                       particles per species per cell there (deposit stress).
    """
    if name == "small_mc64_f64":
        return Problem(name=name, poisson_mode=POISSON_DIRECT)
    if name in ("ec256x512_f32", "mc256x512_f32"):
        return Problem(
            name=name, nr=256, nz=512, lr=0.04, lz=0.08,
            scheme=EC_PIC if name.startswith("ec") else MC_PIC, precision=F32,
            circuit=RESISTOR, v_ext=-500.0, v_fixed=-500.0, r_ext=100.0,
            p_gas=10e-3 * TORR, b_peak=0.05, density=1e16,
            n_per_species=10_000_000, steps=20000, seed=250710728,
            capacity_factor=1.25, poisson_mode=POISSON_DIRECT)
    if name in ("ec512x1024_f32", "mc512x1024_f32", "ec512x1024_clustered_f32"):
        return Problem(
            name=name, nr=512, nz=1024, lr=0.05, lz=0.10,
            scheme=EC_PIC if name.startswith("ec") else MC_PIC, precision=F32,
            circuit=RESISTOR, v_ext=-500.0, v_fixed=-500.0, r_ext=100.0,
            p_gas=20e-3 * TORR, b_peak=0.05, density=1e17,
            n_per_species=50_000_000, steps=20000, seed=250710729,
            capacity_factor=1.1, poisson_mode=POISSON_DIRECT,
            cluster=0.5 if "clustered" in name else 0.0)
    if name in ("magnetron3x3_ec_f32", "magnetron3x3_mc_f32"):
        return Problem(
            name=name, nr=128, nz=128, lr=0.03, lz=0.03, dt=4e-12,
            scheme=EC_PIC if "_ec_" in name else MC_PIC, precision=F32,
            cathode_rmax=0.85 * 0.03, circuit=RESISTOR, v_ext=-300.0, v_fixed=-300.0,
            r_ext=3000.0, gamma_i=0.1, gamma_e=0.1, n_meta=2.5e17, p_gas=10e-3 * TORR,
            density=1e15, te_ev=2.0, n_per_species=200_000, steps=1_000_000,
            seed=250710740, capacity_factor=20.0, poisson_mode=POISSON_MGCG,
            magnets=1)
    raise KeyError(name)


def table1_problems(steps: int, base: str = "magnetron3x3_ec_f32") -> list:
    """The yield / resistance combinations of Table 1 on the 3 x 3 cm
    geometry: ion-induced yield 0.1 or 0.2, R = 3000 or 1000 ohm, electron
    yield 0.1, -300 V source; run k draws random stream k."""
    out = []
    for k, (g, r) in enumerate(((0.1, 3000.0), (0.2, 3000.0), (0.1, 1000.0), (0.2, 1000.0))):
        out.append(preset(base).replace(name=f"{base}_g{g}_r{int(r)}", gamma_i=g, r_ext=r,
                                        run=k, steps=steps))
    return out


ENSEMBLE_GRIDS = (64, 96, 128, 160, 192, 224, 256)
ENSEMBLE_GAMMA = (0.05, 0.1, 0.15, 0.2, 0.3)
ENSEMBLE_R = (10.0, 30.0, 100.0, 300.0, 1000.0)


def ensemble_problems(n_runs: int = 64, scale: float = 1.0, seed: int = 250710732) -> list:
    """The secondary-yield / resistance sweep: n_runs square discharges of
    uneven size.  Cell 312.5 um (domain N x 312.5 um), N from 64 to 256;
    particles per species 1e5 (N / 64)^2 (1e5 to 1.6e6) times `scale`;
    density 1e15 to 1e16 m^-3 (log-spaced over the runs); run k takes yield
    ENSEMBLE_GAMMA[k % 5] and resistance ENSEMBLE_R[(k // 5) % 5], so the 25
    combinations recur over the sizes.  EC-PIC, FP32 state, -500 V source,
    10 mTorr, peak B 0.03 T, dt 5 ps; run k draws the random stream `run = k`."""
    out = []
    for k in range(n_runs):
        n = ENSEMBLE_GRIDS[(k * 3) % len(ENSEMBLE_GRIDS)]
        L = n * 312.5e-6
        dens = 10.0 ** (15.0 + (k % 8) / 7.0)
        npart = max(1000, int(1e5 * (n / 64.0) ** 2 * scale))
        out.append(Problem(
            name=f"sweep{k:02d}", nr=n, nz=n, lr=L, lz=L, scheme=EC_PIC, precision=F32,
            circuit=RESISTOR, v_ext=-500.0, v_fixed=-500.0, r_ext=ENSEMBLE_R[(k // 5) % 5],
            gamma_i=ENSEMBLE_GAMMA[k % 5], p_gas=10e-3 * TORR, b_peak=0.03, density=dens,
            n_per_species=npart, seed=seed, run=k, capacity_factor=1.25, steps=800000))
    return out


def scaled(p: Problem, n_per_species: int) -> Problem:
    """Same discharge with fewer macroparticles (density kept, weight raised)."""
    return p.replace(n_per_species=n_per_species, weight=None)


# ---------------------------------------------------------------------------
# Static magnetron field: one coaxial current loop behind the cathode
# ---------------------------------------------------------------------------

def loop_field(rho, z, a, current=1.0):
    """B of a circular current loop of radius ``a`` in the plane z = 0.

    Closed form with complete elliptic integrals K(m), E(m), m = k^2
    (e.g. Jackson, Classical Electrodynamics, Sec. 5.5; Smythe).  Returns
    (B_rho, B_z) in tesla for ``current`` amperes.
    """
    from scipy.special import ellipe, ellipk

    rho = np.asarray(rho, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    ap2 = (a + rho) ** 2 + z ** 2
    am2 = (a - rho) ** 2 + z ** 2
    m = 4.0 * a * rho / ap2
    kk = ellipk(m)
    ee = ellipe(m)
    c = MU0 * current / (2.0 * np.pi)
    sq = np.sqrt(ap2)
    bz = c / sq * (kk + (a * a - rho * rho - z * z) / am2 * ee)
    with np.errstate(invalid="ignore", divide="ignore"):
        br = c * z / (rho * sq) * (-kk + (a * a + rho * rho + z * z) / am2 * ee)
    br = np.where(rho > 0.0, br, 0.0)
    return br, bz


def magnetron_field(p: Problem):
    """Nodal (B_r, B_z), each (nz+1)*(nr+1) flat, r fastest.

    A single loop of radius 0.45*L_r placed 0.15*L_r behind the cathode plane,
    scaled so that max |B| over the z = 0 node row equals ``b_peak``.
    """
    r = np.arange(p.nr + 1) * p.dr
    z = np.arange(p.nz + 1) * p.dz
    a = 0.45 * p.lr
    z0 = -0.15 * p.lr
    R, Z = np.meshgrid(r, z)  # shape (nz+1, nr+1)
    br, bz = loop_field(R, Z - z0, a)
    mag0 = np.sqrt(br[0] ** 2 + bz[0] ** 2).max()
    s = p.b_peak / mag0 if mag0 > 0 else 0.0
    return (np.ascontiguousarray((br * s).ravel()),
            np.ascontiguousarray((bz * s).ravel()))


def magnetized_cylinder_field(rho, z, a, z_bot, z_top, br_tesla, nquad=96):
    """B of a cylinder of radius ``a`` uniformly magnetised along z (remanent
    flux density ``br_tesla``, i.e. mu0 M) between z_bot and z_top.

    The magnetisation is equivalent to an azimuthal surface current M per
    unit length on the curved face (a finite solenoid), so the field is the
    current-loop field integrated over the height (Gauss-Legendre, nquad
    points).  Valid outside the magnet.  Returns (B_rho, B_z) in tesla.
    """
    x, wq = np.polynomial.legendre.leggauss(nquad)
    zs = 0.5 * (z_top - z_bot) * x + 0.5 * (z_top + z_bot)
    k_per_m = br_tesla / MU0            # M = surface current per unit length
    br = np.zeros(np.broadcast(rho, z).shape)
    bz = np.zeros_like(br)
    for zq, wk in zip(zs, wq):
        r_, z_ = loop_field(rho, z - zq, a, current=1.0)
        f = 0.5 * (z_top - z_bot) * wk * k_per_m
        br += f * r_
        bz += f * z_
    return br, bz


def two_magnet_field(p: Problem, br_tesla=1.1, inner_radius=6.5e-3, outer_r0=0.017,
                     outer_width=2e-3, top=-2e-3, height=10e-3):
    """Nodal (B_r, B_z) of the unbalanced (type II) two-magnet layout of
    Section 3: an inner cylinder of radius 6.5 mm and an outer ring at
    L_1 = 1.7 cm, 2 mm wide, both magnetised at 1.1 T with opposite
    polarity (outer to inner flux ratio (1.9^2 - 1.7^2) / 0.65^2 = 1.70).
    Section 3 does not give the magnets' height or depth; they are taken
    10 mm tall with their faces 2 mm behind the cathode plane.  The field is
    that of the magnets in free space (equivalent surface currents), which is
    what the paper's scalar-potential solve on an enlarged domain
    approximates."""
    r = np.arange(p.nr + 1) * p.dr
    z = np.arange(p.nz + 1) * p.dz
    R, Z = np.meshgrid(r, z)
    zb, zt = top - height, top
    b_in = magnetized_cylinder_field(R, Z, inner_radius, zb, zt, br_tesla)
    b_o2 = magnetized_cylinder_field(R, Z, outer_r0 + outer_width, zb, zt, -br_tesla)
    b_o1 = magnetized_cylinder_field(R, Z, outer_r0, zb, zt, br_tesla)
    br = b_in[0] + b_o2[0] + b_o1[0]
    bz = b_in[1] + b_o2[1] + b_o1[1]
    return np.ascontiguousarray(br.ravel()), np.ascontiguousarray(bz.ravel())


# ---------------------------------------------------------------------------
# Electron-argon cross sections (analytic fits; project-defined)
# ---------------------------------------------------------------------------

N_TABLE = 20001
DE_TABLE = 0.05  # eV


def cross_sections(e_exc=11.5, e_iz=15.76, n=N_TABLE, de=DE_TABLE, e_iz_meta=4.20):
    """Tabulated cross sections (m^2) at E_k = k*de eV, k = 0..n-1.

    Rows: elastic, excitation, ionization from the ground state, ionization
    from the metastable Ar* (Section 3's processes (1a)-(1d)).  Smooth
    analytic forms in the magnitude range of e-Ar data: an elastic curve
    peaking near 10-15 eV, a Thomson-like excitation and Lotz ionization
    (ground state: 6 outer electrons at 15.76 eV; metastable: the one excited
    electron at 4.20 eV).  The inelastic forms vanish at and below threshold.
    """
    e = np.arange(n, dtype=np.float64) * de
    el = 1.5e-19 * (e / 12.0) ** 1.2 / (1.0 + (e / 12.0) ** 2.2) + 2.0e-21
    el = el + 1.0e-20 / (1.0 + e)  # low-energy floor
    x = np.where(e > e_exc, e / e_exc, 1.0)
    ex = np.where(e > e_exc, 3.0e-20 * np.log(x) / x, 0.0)
    # Lotz: sigma = a q ln(E/I) / (E I), a = 4.5e-18 eV^2 m^2, q outer electrons
    y = np.where(e > e_iz, e, e_iz)
    iz = np.where(e > e_iz, 4.5e-18 * 6.0 * np.log(y / e_iz) / (y * e_iz), 0.0)
    ym = np.where(e > e_iz_meta, e, e_iz_meta)
    izm = np.where(e > e_iz_meta, 4.5e-18 * 1.0 * np.log(ym / e_iz_meta) / (ym * e_iz_meta), 0.0)
    return np.ascontiguousarray(np.stack([el, ex, iz, izm]))


# ---------------------------------------------------------------------------
# Initial load (paper, Section 4: seed population of uniform-density e-, Ar+)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class SpeciesArrays:
    r: np.ndarray
    z: np.ndarray
    vr: np.ndarray
    vt: np.ndarray
    vz: np.ndarray
    id: np.ndarray  # uint32

    @property
    def n(self):
        return int(self.r.shape[0])

    def copy(self):
        return SpeciesArrays(*(a.copy() for a in
                               (self.r, self.z, self.vr, self.vt, self.vz, self.id)))


def load_uniform(p: Problem, n: Optional[int] = None, seed_offset: int = 0):
    """Uniform-in-volume positions (r = R sqrt(U), z = L U) and Maxwellian
    velocities (Te for electrons, Ti for ions); ids 0..N-1 per species.
    Sampled velocities are taken as v^{n-1/2}.  With p.cluster = c > 0 the
    first round(c N) particles of each species are instead uniform in volume
    over the ring 0.35 R < r < 0.5 R, 0 <= z < 0.1 L.
    """
    n = p.n_per_species if n is None else n
    rng = np.random.Generator(np.random.PCG64(p.seed + 7919 * seed_offset))
    out = []
    for s, t_ev in ((0, p.te_ev), (1, p.ti_ev)):
        m = M_E if s == 0 else (M_AR - M_E)
        vth = math.sqrt(t_ev * E_CHARGE / m)
        r = p.lr * np.sqrt(rng.random(n))
        z = p.lz * rng.random(n)
        nc = int(round(p.cluster * n))
        if nc > 0:
            r0, r1 = 0.35 * p.lr, 0.5 * p.lr
            r[:nc] = np.sqrt(r0 * r0 + (r1 * r1 - r0 * r0) * rng.random(nc))
            z[:nc] = 0.1 * p.lz * rng.random(nc)
        # keep strictly inside [0, L): rng.random() < 1 already
        v = rng.standard_normal((3, n)) * vth
        out.append(SpeciesArrays(r, z, v[0].copy(), v[1].copy(), v[2].copy(),
                                 np.arange(n, dtype=np.uint32)))
    return out


def thermal_box(nr: int, nz: int, cell: float, ppc: int, scheme: int, precision: int = F32,
                seed: int = 99):
    """Closed box for the EC-/MC-PIC energy comparison (Sections 2 and 5):
    nr x nz cells of size `cell`, the cell three Debye lengths at Te = 2 eV
    (density set to match), dt = 0.1 / w_pe, reflecting grounded walls, no
    collisions, emission or magnetic field, frozen cold ions, electrons
    started on the ions' positions (quiet, neutral); ppc particles per species
    per cell.  Returns (problem, [electrons, ions])."""
    eps0 = 8.8541878128e-12
    te = 2.0
    lam = cell / 3.0
    n0 = eps0 * te / (E_CHARGE * lam * lam)
    wpe = math.sqrt(n0 * E_CHARGE * E_CHARGE / (eps0 * M_E))
    p = Problem(name=f"box{nr}x{nz}", nr=nr, nz=nz, lr=nr * cell, lz=nz * cell,
                circuit=FIXED_V, v_fixed=0.0, v_ext=0.0, mcc_on=0, see_on=0, frozen_ions=1,
                wall_bc=(REFLECT, REFLECT, REFLECT), gamma_i=0.0, b_peak=0.0, scheme=scheme,
                precision=precision, dt=0.1 / wpe, density=n0, n_per_species=nr * nz * ppc,
                te_ev=te, ti_ev=0.0, seed=seed)
    el, io = load_uniform(p)
    io.vr[:] = 0.0
    io.vt[:] = 0.0
    io.vz[:] = 0.0
    el.r[:] = io.r
    el.z[:] = io.z
    return p, [el, io]


def inputs(p: Problem, n: Optional[int] = None):
    """Everything a run needs: (B_r, B_z, sigma table, [electrons, ions])."""
    br, bz = two_magnet_field(p) if p.magnets == 1 else magnetron_field(p)
    sig = cross_sections(p.e_exc, p.e_iz, e_iz_meta=p.e_iz_meta)
    parts = load_uniform(p, n)
    return br, bz, sig, parts
