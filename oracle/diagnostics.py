"""Plasma diagnostics of the oracle: plain FP64 numpy, written from the
definitions the paper gives.  Test infrastructure: only the tests, the smoke
check and the benchmark's CPU-baseline leg use this module.

Readings (the paper names the quantities, not their discretisation):

* Cell moments (Section 5, electron temperature from the second moment of
  the particle data): particles are binned by cell (nearest grid point,
  cell (i, j) holds dr i <= r < dr (i + 1), dz j <= z < dz (j + 1)); per
  cell the count N, the velocity sum S1 and the sum of squared speeds S2.
* Cell density n = N w / V_cell with V_cell = pi (r_{i+1}^2 - r_i^2) dz;
  cell temperature T = m (S2 / N - |S1 / N|^2) / (3 e) in eV (cells with
  fewer than two particles have none); Debye length
  lambda_D = sqrt(eps0 T / (e n_e)).
* The Debye length that is compared with the cell size is the one where the
  electron density is largest (Section 4): the cell of maximum n_e.
* Axial profiles over a radial band r0 <= r_c < r1 of cell centres
  (Section 5 uses 1.0 cm < r < 1.5 cm): band densities per cell row
  (counts times w over band volume) and the band potential per node row
  (mean over the band cells of the midpoint of each cell's lower edge),
  whose difference gives E_z per cell row.
* Sheath edge (Section 4): where n_e = n_i / 2, the first cell row from the
  cathode with n_e >= n_i / 2, interpolated linearly between cell centres
  from the row below (0 if the first row already satisfies it).  Bulk
  (Section 4): where E_z = 0 above the sheath edge, the first sign change of
  E_z from negative to non-negative, interpolated between cell centres.
* Region temperature (Section 5): over the band cells whose centre lies in
  the region (sheath below the sheath edge, pre-sheath between the edges,
  bulk above the bulk edge), the count-weighted mean of the cell
  temperatures.
* Re-weighting (Section 5 removes particles and triples the weight; read as
  keeping one particle in three, the ones whose id is a multiple of 3, and
  tripling the weight, which keeps the expected charge).
"""
import math

import numpy as np

QE = 1.602176634e-19
EPS0 = 8.8541878128e-12


def cell_index(p, r, z):
    """Cell of each position: i = floor(r / dr), j = floor(z / dz), clamped
    to the grid."""
    i = np.minimum(np.floor(np.asarray(r) / p.dr).astype(np.int64), p.nr - 1)
    j = np.minimum(np.floor(np.asarray(z) / p.dz).astype(np.int64), p.nz - 1)
    return np.maximum(i, 0), np.maximum(j, 0)


def cell_moments(p, i, j, vr, vt, vz):
    """Per cell (arrays of shape (nz, nr)): count N, velocity sums S1 (3, nz,
    nr) and the sum of squared speeds S2."""
    c = np.asarray(j, np.int64) * p.nr + np.asarray(i, np.int64)
    nc = p.nr * p.nz
    n = np.bincount(c, minlength=nc).astype(np.float64)
    s1 = np.stack([np.bincount(c, weights=np.asarray(v, np.float64), minlength=nc)
                   for v in (vr, vt, vz)])
    v2 = (np.asarray(vr, np.float64) ** 2 + np.asarray(vt, np.float64) ** 2
          + np.asarray(vz, np.float64) ** 2)
    s2 = np.bincount(c, weights=v2, minlength=nc)
    return n.reshape(p.nz, p.nr), s1.reshape(3, p.nz, p.nr), s2.reshape(p.nz, p.nr)


def cell_volumes(p):
    r = np.arange(p.nr + 1) * p.dr
    v = math.pi * (r[1:] ** 2 - r[:-1] ** 2) * p.dz
    return np.broadcast_to(v, (p.nz, p.nr))


def cell_temperature(m, n, s1, s2):
    """T (eV) per cell from its moments; 0 where fewer than two particles."""
    with np.errstate(invalid="ignore", divide="ignore"):
        mean2 = s2 / n - (s1[0] ** 2 + s1[1] ** 2 + s1[2] ** 2) / (n * n)
        t = m * mean2 / (3.0 * QE)
    return np.where(n >= 2, np.maximum(t, 0.0), 0.0)


def plasma_maps(p, mom_e, n_i_count):
    """Cell maps: n_e, n_i (m^-3), T_e (eV) and lambda_D (m; inf where
    n_e or T_e is zero)."""
    sp = p.species()
    w = sp[0][2]
    vol = cell_volumes(p)
    n_e = mom_e[0] * w / vol
    n_i = n_i_count * sp[1][2] / vol
    te = cell_temperature(sp[0][1], *mom_e)
    with np.errstate(invalid="ignore", divide="ignore"):
        lam = np.where((n_e > 0) & (te > 0), np.sqrt(EPS0 * te / (QE * n_e)), np.inf)
    return n_e, n_i, te, lam


def band_cells(p, r0, r1):
    rc = (np.arange(p.nr) + 0.5) * p.dr
    return (rc >= r0) & (rc < r1)


def locate(p, mom_e, n_i_count, phi, r0, r1):
    """Sheath edge, bulk edge and the three region temperatures over the band
    r0 <= r_c < r1.  Returns a dict; an edge that is not found is NaN."""
    sp = p.species()
    band = band_cells(p, r0, r1)
    vol = cell_volumes(p)[:, band].sum(axis=1)
    ne = mom_e[0][:, band].sum(axis=1) * sp[0][2] / vol
    ni = n_i_count[:, band].sum(axis=1) * sp[1][2] / vol
    ph = np.asarray(phi, np.float64).reshape(p.nz + 1, p.nr + 1)
    idx = np.nonzero(band)[0]
    pbar = 0.5 * (ph[:, idx] + ph[:, idx + 1]).mean(axis=1)      # per node row
    ez = -(pbar[1:] - pbar[:-1]) / p.dz                          # per cell row
    zc = (np.arange(p.nz) + 0.5) * p.dz
    f = ne - 0.5 * ni
    z_s = math.nan
    js = None
    for j in range(p.nz):
        if f[j] >= 0:
            js = j
            z_s = 0.0 if j == 0 else zc[j - 1] + p.dz * f[j - 1] / (f[j - 1] - f[j])
            break
    z_b = math.nan
    if js is not None:
        for j in range(max(js, 1), p.nz):
            if ez[j - 1] < 0 <= ez[j]:
                z_b = zc[j - 1] + p.dz * (-ez[j - 1]) / (ez[j] - ez[j - 1])
                break
    te = cell_temperature(sp[0][1], *mom_e)[:, band]
    n = mom_e[0][:, band]
    use = n >= 2
    rows = np.broadcast_to(zc[:, None], te.shape)
    if math.isnan(z_s):
        region = np.zeros(te.shape, np.int64)
    else:
        region = np.where(rows < z_s, 0, 1)
        if not math.isnan(z_b):
            region = np.where(rows >= z_b, 2, region)
    t_reg, n_reg = [], []
    for k in range(3):
        m = use & (region == k)
        nk = n[m].sum()
        n_reg.append(int(nk))
        t_reg.append(float((n[m] * te[m]).sum() / nk) if nk > 0 else 0.0)
    return {"z_sheath": z_s, "z_bulk": z_b, "te_region": t_reg, "n_region": n_reg,
            "ne_profile": ne, "ni_profile": ni, "ez_profile": ez}


def debye_at_peak(p, maps):
    """lambda_D, n_e and T_e in the cell of largest electron density (first
    such cell in j-major order)."""
    n_e, n_i, te, lam = maps
    k = int(np.argmax(n_e))
    j, i = divmod(k, p.nr)
    return {"lambda_d": float(lam[j, i]), "n_e": float(n_e[j, i]), "te": float(te[j, i]),
            "cell": (i, j)}


def reweight_keep(ids, k):
    """Particles kept by the re-weighting: those whose id is a multiple of k."""
    return (np.asarray(ids, np.uint64) % np.uint64(k)) == 0
