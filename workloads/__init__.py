"""Seeded synthetic inputs shaped like the paper's synthesis workloads.

This module only draws inputs: a 72-depth model atmosphere, a line list, a
log-uniform wavelength grid and the fitted corrections.  It holds none of the
synthesis arithmetic (populations, opacity, transfer), so the CPU oracle and
the GPU path can both consume its output without sharing any method code.

Recipes (all numbers are the workload definitions, not physics of the path):

* Grid (Sec. 2.1, Eqs. 1-2): lambda_i = lambda_first (1 + 1/R)^i with
  N = floor(ln(lambda_max/lambda_min) / ln(1 + 1/R)) + 1 samples.
* Atmosphere: column mass m_j = 10^(-3 + 4 j/71) g cm^-2; grey temperature
  T = Teff [0.75 (tau + 2/3)]^(1/4) with tau = kappa0 m (the grey law of
  Sec. 4, Eq. 26); n_H = g m / (1.1 k Teff) (hydrostatic equilibrium, Sec. 3
  Eq. 10, with P_rad = P_0 = 0 and He/H = 0.1); n_e = 1e-4 g m^0.8/(1.1 k Teff);
  n_pert = n_H; rho = 1.4 m_u n_H.  Power-law continuum kappa0 (lambda /
  lambda_ref)^alpha with kappa0 = 1 cm^2 g^-1, alpha = -1, lambda_ref the
  geometric middle of the window.
* Species: mass ~ U[12, 60] amu, log abundance ~ U[-8, -4] relative to H,
  ionisation energy ~ U[5, 9] eV, partition functions U_I, U_II ~ U{1..10}
  (constant with depth).  "Molecular" species carry an infinite ionisation
  energy (single stage).
* Lines: log gf ~ U[-4, 0], E ~ U[0, 6] eV, ion stage ~ Bernoulli(1/2),
  log gamma_rad ~ U[7, 9] s^-1, log gamma_S ~ U[-7, -4] and
  log gamma_vdW ~ U[-9, -7] cm^3 s^-1 (Table 1 line and broadening symbols).

Seeds: numpy PCG64, one fixed seed per workload (240001-240006); star b of the batch
workload uses 250000 + b.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

K_BOLTZ = 1.380649e-16     # erg/K  (CODATA 2018, exact)
AMU_G = 1.66053906660e-24  # g

N_DEPTH = 72
WINDOW_NM = 0.3


@dataclasses.dataclass
class Grid:
    lam_first_nm: float
    R: float
    N: int


@dataclasses.dataclass
class Atmosphere:
    T: np.ndarray          # [D] K
    m: np.ndarray          # [D] g cm^-2, strictly increasing inward
    ne: np.ndarray         # [D] cm^-3
    npert: np.ndarray      # [D] cm^-3
    rho: np.ndarray        # [D] g cm^-3
    n_species: np.ndarray  # [S, D] element (species) totals, cm^-3
    chi_ion_eV: np.ndarray  # [S] (inf => single stage)
    U: np.ndarray          # [S, 2, D] partition functions
    mass_amu: np.ndarray   # [S]
    kappa0: float = 1.0    # cm^2 g^-1
    lam_ref_nm: float = 500.0
    alpha: float = -1.0
    sigma_c: np.ndarray = None   # [D] continuum scattering per unit mass at lam_ref (None: no scattering)
    sigma_alpha: float = 0.0     # sigma_c(lambda) = sigma_c (lambda / lam_ref)^sigma_alpha

    @property
    def D(self):
        return int(self.T.shape[0])

    @property
    def S(self):
        return int(self.mass_amu.shape[0])


@dataclasses.dataclass
class LineList:
    lam0_nm: np.ndarray    # [L] float64
    loggf: np.ndarray      # [L]
    E_eV: np.ndarray       # [L]
    species: np.ndarray    # [L] int32
    ion: np.ndarray        # [L] int32 (0 neutral, 1 singly ionised)
    log_grad: np.ndarray   # [L] log10 s^-1
    log_gstark: np.ndarray  # [L] log10 cm^3 s^-1
    log_gvdw: np.ndarray   # [L] log10 cm^3 s^-1

    @property
    def L(self):
        return int(self.lam0_nm.shape[0])

    def take(self, idx):
        return LineList(*[getattr(self, f.name)[idx] for f in dataclasses.fields(self)])


@dataclasses.dataclass
class Params:
    dgf: np.ndarray    # [L] dex
    ddamp: np.ndarray  # [L] dex (scales the total damping width)
    dA: np.ndarray     # [S] dex
    xi_kms: float
    ddamp_family: np.ndarray = None   # [3, L] dex per damping family (radiative, Stark, van der Waals), or None


@dataclasses.dataclass
class Workload:
    name: str
    grid: Grid
    atm: Atmosphere
    lines: LineList
    params: Params
    window_nm: float = WINDOW_NM
    quadrature: str = "gauss3"
    center_eta: float = 0.0          # continuum-referenced centre test threshold (0: off)
    extra: dict = dataclasses.field(default_factory=dict)


def grid_for(lam_min, lam_max, R):
    h = math.log1p(1.0 / R)
    N = int(math.floor(math.log(lam_max / lam_min) / h)) + 1
    return Grid(float(lam_min), float(R), N)


def grid_last(grid):
    return grid.lam_first_nm * (1.0 + 1.0 / grid.R) ** (grid.N - 1)


def make_atmosphere(rng, Teff, logg, S, n_molecular=0, metal_shift=0.0, lam_ref_nm=500.0,
                    D=N_DEPTH):
    g = 10.0 ** logg
    j = np.arange(D, dtype=np.float64)
    m = 10.0 ** (-3.0 + 4.0 * j / (D - 1))
    kappa0 = 1.0
    tau = kappa0 * m
    T = Teff * (0.75 * (tau + 2.0 / 3.0)) ** 0.25
    scale = g / (1.1 * K_BOLTZ * Teff)
    nH = scale * m
    ne = 1e-4 * scale * m ** 0.8
    rho = 1.4 * AMU_G * nH
    mass = rng.uniform(12.0, 60.0, S)
    logA = rng.uniform(-8.0, -4.0, S) + metal_shift
    chi = rng.uniform(5.0, 9.0, S)
    Uc = rng.integers(1, 11, size=(S, 2)).astype(np.float64)
    if n_molecular:
        mol = np.arange(S - n_molecular, S)
        mass[mol] = np.array([26.0, 28.0, 30.0, 32.0][:n_molecular])
        chi[mol] = np.inf
    U = np.repeat(Uc[:, :, None], D, axis=2)
    n_species = (10.0 ** logA)[:, None] * nH[None, :]
    return Atmosphere(T=T, m=m, ne=ne, npert=nH.copy(), rho=rho, n_species=n_species,
                      chi_ion_eV=chi, U=U, mass_amu=mass, kappa0=kappa0,
                      lam_ref_nm=float(lam_ref_nm), alpha=-1.0)


def _damping(rng, n):
    return (rng.uniform(7.0, 9.0, n), rng.uniform(-7.0, -4.0, n), rng.uniform(-9.0, -7.0, n))


def atomic_lines(rng, n, lam_lo, lam_hi, n_atomic_species, loggf=None, E_max=6.0, lam0=None):
    if lam0 is None:
        lam0 = rng.uniform(lam_lo, lam_hi, n)
    if loggf is None:
        loggf = rng.uniform(-4.0, 0.0, n)
    E = rng.uniform(0.0, E_max, n)
    sp = rng.integers(0, n_atomic_species, n).astype(np.int32)
    ion = rng.integers(0, 2, n).astype(np.int32)
    gr, gs, gw = _damping(rng, n)
    return LineList(lam0.astype(np.float64), loggf, E, sp, ion, gr, gs, gw)


def band_lines(rng, n_bands, per_band, lam_lo, lam_hi, mol_species):
    """Regularly spaced band-like sequences of 'molecular' lines."""
    lam, sp = [], []
    width = lam_hi - lam_lo
    for _ in range(n_bands):
        dmax = min(0.05, 0.999 * width / per_band)
        dlam = rng.uniform(min(0.01, dmax), dmax)
        head = rng.uniform(lam_lo, lam_hi - dlam * (per_band - 1))
        lam.append(head + dlam * np.arange(per_band))
        sp.append(np.full(per_band, rng.choice(mol_species), dtype=np.int32))
    n = n_bands * per_band
    lam = np.concatenate(lam) if lam else np.zeros(0)
    sp = np.concatenate(sp) if sp else np.zeros(0, np.int32)
    loggf = rng.normal(-2.0, 1.0, n)
    E = rng.uniform(0.0, 2.0, n)
    gr, gs, gw = _damping(rng, n)
    return LineList(lam.astype(np.float64), loggf, E, sp, np.zeros(n, np.int32), gr, gs, gw)


def concat_lines(a, b):
    return LineList(*[np.concatenate([getattr(a, f.name), getattr(b, f.name)])
                      for f in dataclasses.fields(LineList)])


def zero_params(L, S, xi):
    return Params(np.zeros(L), np.zeros(L), np.zeros(S), float(xi))


def solar_500_503nm(seed=240_001):
    """Plain forward: 500-503 nm, R=300,000, solar, 1,000 lines, 10 species."""
    rng = np.random.Generator(np.random.PCG64(seed))
    grid = grid_for(500.0, 503.0, 3.0e5)
    lam_ref = math.sqrt(500.0 * 503.0)
    atm = make_atmosphere(rng, 5777.0, 4.44, 10, lam_ref_nm=lam_ref)
    lines = atomic_lines(rng, 1000, 500.0, 503.0, 10)
    return Workload("500-503nm_R3e5_L1e3_solar", grid, atm, lines, zero_params(1000, 10, 0.7))


def _apogee_mixture(rng, L, lam_lo, lam_hi, S_atomic, mol_species):
    n_band_lines = int(round(0.3 * L / 600.0)) * 600
    atom = atomic_lines(rng, L - n_band_lines, lam_lo, lam_hi, S_atomic)
    bands = band_lines(rng, n_band_lines // 600, 600, lam_lo, lam_hi, mol_species)
    return concat_lines(atom, bands)


def giant_1500_1700nm(seed=240_002, L=200_000):
    """1500-1700 nm, R=300,000, Arcturus-like giant, 2e5 lines (30% in bands)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    grid = grid_for(1500.0, 1700.0, 3.0e5)
    lam_ref = math.sqrt(1500.0 * 1700.0)
    atm = make_atmosphere(rng, 4500.0, 2.5, 20, n_molecular=2, lam_ref_nm=lam_ref)
    lines = _apogee_mixture(rng, L, 1500.0, 1700.0, 18, [18, 19])
    return Workload("1500-1700nm_R3e5_L2e5_giant", grid, atm, lines,
                    zero_params(lines.L, 20, 1.7))


def solar_300_1000nm(seed=240_003, L=5_000_000):
    """300-1000 nm, R=300,000, solar, 5e6 lines with density ~ lambda^-2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = 300.0, 1000.0
    grid = grid_for(lo, hi, 3.0e5)
    atm = make_atmosphere(rng, 5777.0, 4.44, 40, lam_ref_nm=math.sqrt(lo * hi))
    u = rng.uniform(0.0, 1.0, L)
    lam0 = 1.0 / (1.0 / lo - u * (1.0 / lo - 1.0 / hi))
    loggf = rng.normal(-2.5, 1.2, L)
    lines = atomic_lines(rng, L, lo, hi, 40, loggf=loggf, lam0=lam0)
    return Workload("300-1000nm_R3e5_L5e6_solar", grid, atm, lines, zero_params(L, 40, 0.7))


def giant_1500_1700nm_fit(seed=240_004):
    """Differentiation on the 1500-1700 nm workload: truth perturbation + noise."""
    wl = giant_1500_1700nm()
    rng = np.random.Generator(np.random.PCG64(seed))
    L, S = wl.lines.L, wl.atm.S
    truth = Params(rng.normal(0.0, 0.05, L), rng.normal(0.0, 0.1, L), rng.normal(0.0, 0.05, S),
                   wl.params.xi_kms + 0.2)
    sigma = 0.01
    noise = rng.normal(0.0, sigma, wl.grid.N)
    wl.name = "1500-1700nm_R3e5_L2e5_giant_fwdbwd"
    wl.extra = dict(truth=truth, sigma=sigma, noise=noise)
    return wl


BATCH_N_MAX = None  # set per star from the 1500-1700 nm interval


def batch_star(b, seed_base=250_000, S=20):
    """Star b of the 256-star batch (window and line count drawn per star)."""
    rng = np.random.Generator(np.random.PCG64(seed_base + b))
    Teff = rng.uniform(3500.0, 7000.0)
    logg = rng.uniform(1.0, 5.0)
    feh = rng.uniform(-2.0, 0.5)
    xi = rng.uniform(0.5, 2.5)
    R = 3.0e5
    full = grid_for(1500.0, 1700.0, R)
    Nb = int(rng.integers(5000, 40001))
    clamped = Nb > full.N
    Nb = min(Nb, full.N)
    i0 = int(rng.integers(0, full.N - Nb + 1))
    lam_first = 1500.0 * (1.0 + 1.0 / R) ** i0
    grid = Grid(lam_first, R, Nb)
    lam_last = grid_last(grid)
    Lb = int(rng.integers(10_000, 200_001))
    atm = make_atmosphere(rng, Teff, logg, S, n_molecular=2, metal_shift=feh,
                          lam_ref_nm=math.sqrt(lam_first * lam_last))
    lines = _apogee_mixture(rng, Lb, lam_first, lam_last, S - 2, [S - 2, S - 1])
    wl = Workload("batch_star_%d" % b, grid, atm, lines, zero_params(lines.L, S, xi))
    wl.extra = dict(Teff=Teff, logg=logg, feh=feh, clamped=clamped)
    return wl


def batch_stars(n_star=256):
    return [batch_star(b) for b in range(n_star)]


def tiny(seed=7, L=12, N=400, D=8, S=3, lam_lo=500.0, R=3.0e5, xi=1.0, window_nm=WINDOW_NM,
         logg=4.44, Teff=5777.0, n_molecular=0):
    """Small random case for brute-force and closed-form checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    grid = Grid(lam_lo, R, N)
    lam_hi = grid_last(grid)
    atm = make_atmosphere(rng, Teff, logg, S, n_molecular=n_molecular,
                          lam_ref_nm=math.sqrt(lam_lo * lam_hi), D=D)
    lines = atomic_lines(rng, L, lam_lo, lam_hi, S - n_molecular)
    if n_molecular:
        lines.species[::3] = S - 1
        lines.ion[::3] = 0
    wl = Workload("tiny_%d" % seed, grid, atm, lines, zero_params(L, S, xi), window_nm=window_nm)
    return wl


def random_params(rng, L, S, xi, scale=1.0):
    return Params(rng.normal(0.0, 0.05 * scale, L), rng.normal(0.0, 0.1 * scale, L),
                  rng.normal(0.0, 0.05 * scale, S), float(xi))




def apogee_instrument(grid, R_lsf=(20000.0, 25000.0), vb_max_kms=20.0):
    """Observed pixels and LSF widths standing in for an APOGEE-like spectrograph
    on the 1500-1700 nm grid: log-uniform pixels with d(log10 lambda) = 6e-6 over
    1514-1696 nm in three detector ranges (gaps 1581-1585 and 1644-1647 nm), and
    a Gaussian LSF whose resolving power runs linearly from R_lsf[0] to R_lsf[1]
    across the range (sigma in ln lambda = 1 / (2 sqrt(2 ln 2) R)).  The
    calibration-derived LSF of the paper is not available."""
    dln = 6.0e-6 * math.log(10.0)
    x = np.arange(math.log(1514.0), math.log(1696.0), dln)
    lam = np.exp(x)
    keep = ~(((lam > 1581.0) & (lam < 1585.0)) | ((lam > 1644.0) & (lam < 1647.0)))
    lam = lam[keep]
    lo, hi = grid.lam_first_nm, grid_last(grid)
    R = R_lsf[0] + (R_lsf[1] - R_lsf[0]) * (lam - lam[0]) / (lam[-1] - lam[0])
    sigma_ln = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)) * R)
    assert lam[0] > lo and lam[-1] < hi
    return lam, sigma_ln, vb_max_kms


# ------------------------------------------------------------ line calibration
CM1_EV = 1.239841984e-4        # one wavenumber (cm^-1) in eV
CAL_RECORDS = 42_886           # atomic records of the 1500-1700 nm calibration interval
CAL_DE_CM = 2.0                # grouping tolerance in lower-level energy, cm^-1
CAL_DLAM_NM = 0.035            # grouping tolerance in wavelength, nm
CAL_TRUTH_SIGMA = (0.1, 0.3, 0.3, 0.2)   # dex: log gf, radiative, Stark, van der Waals


def complex_lines(rng, n, lam_lo, lam_hi, n_species, mean_extra=0.7, dlam_nm=0.012, dE_cm=0.7):
    """n atomic records arranged in complexes (stand-ins for fine-structure,
    hyperfine and isotopic components): a complex has 1 + Poisson(mean_extra)
    components sharing its species and ion stage, each within +-dlam_nm of the
    complex wavelength and +-dE_cm of its lower-level energy, with log gf =
    complex value + N(0, 0.3).  Complex wavelength, energy, log gf, species and
    ion follow the atomic recipe.  Returns (LineList, complex id per record)."""
    est = int(n / (1.0 + mean_extra) * 1.3) + 16
    ks = 1 + rng.poisson(mean_extra, est)
    cs = np.cumsum(ks)
    nc = int(np.searchsorted(cs, n)) + 1
    ks = ks[:nc].copy()
    ks[-1] -= int(cs[nc - 1] - n)
    cid = np.repeat(np.arange(nc), ks)
    lam_c = rng.uniform(lam_lo, lam_hi, nc)
    E_c = rng.uniform(0.0, 6.0, nc)
    gf_c = rng.uniform(-4.0, 0.0, nc)
    sp_c = rng.integers(0, n_species, nc).astype(np.int32)
    ion_c = rng.integers(0, 2, nc).astype(np.int32)
    lam = lam_c[cid] + rng.uniform(-dlam_nm, dlam_nm, n)
    E = np.maximum(E_c[cid] + rng.uniform(-dE_cm, dE_cm, n) * CM1_EV, 0.0)
    loggf = gf_c[cid] + rng.normal(0.0, 0.3, n)
    gr, gs, gw = _damping(rng, n)
    return LineList(lam, loggf, E, sp_c[cid], ion_c[cid], gr, gs, gw), cid


def telluric_weights(rng, lam_nm, n_features, mask_below=0.5):
    """Relative pixel weights from a synthetic telluric transmission:
    T = exp(-sum_k d_k exp(-((lambda - lambda_k) / w_k)^2 / 2)) with
    d_k ~ U[0.02, 1.5], w_k ~ U[0.005, 0.03] nm; weight T where T >= mask_below,
    else 0 (masked)."""
    lam_nm = np.asarray(lam_nm, np.float64)
    tau = np.zeros(lam_nm.size)
    c = rng.uniform(lam_nm[0], lam_nm[-1], n_features)
    d = rng.uniform(0.02, 1.5, n_features)
    w = rng.uniform(0.005, 0.03, n_features)
    for ck, dk, wk in zip(c, d, w):
        a, b = np.searchsorted(lam_nm, [ck - 6.0 * wk, ck + 6.0 * wk])
        tau[a:b] += dk * np.exp(-0.5 * ((lam_nm[a:b] - ck) / wk) ** 2)
    T = np.exp(-tau)
    return np.where(T >= mask_below, T, 0.0)


def _atlas_pixels(grid, step_px, margin_px, R_atlas):
    """Observed pixels every step_px native pixels, margin_px in from the grid
    ends, with a Gaussian LSF of resolving power R_atlas (an FTS-like atlas)."""
    h = math.log1p(1.0 / grid.R)
    x0 = math.log(grid.lam_first_nm)
    x = x0 + h * np.arange(margin_px, grid.N - 1 - margin_px, step_px)
    sigma = np.full(x.size, 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)) * R_atlas))
    return np.exp(x), sigma


@dataclasses.dataclass
class CalStandard:
    """One standard spectrum of the calibration: its workload (shared grid and
    line list), observed pixels, LSF widths, velocities, weights w and c."""
    name: str
    wl: Workload
    lam_obs_nm: np.ndarray
    lsf_sigma_ln: np.ndarray
    vb_max_kms: float
    vel: tuple
    w: np.ndarray
    c: float


@dataclasses.dataclass
class CalWorkload:
    name: str
    grid: Grid
    lines: LineList
    active: np.ndarray            # [L] bool: atomic records that are calibrated
    complex_id: np.ndarray        # [n_records] complex of each atomic record
    standards: list


# (name, Teff, log g, [M/H], xi km/s, Gaussian dispersion km/s, epochs): Sec. 6
CAL_STARS = (("sun", 5777.0, 4.44, 0.0, 0.7, 1.55, 1), ("arcturus", 4286.0, 1.66, -0.52, 1.7, 2.5, 2))


def _cal_standards(rng, grid, lines, S, D, species_seed, steps, R_atlas, margin, n_tell):
    lam_ref = math.sqrt(grid.lam_first_nm * grid_last(grid))
    out = []
    for (name, Teff, logg, feh, xi, vb, n_ep), step in zip(CAL_STARS, steps):
        atm = make_atmosphere(np.random.Generator(np.random.PCG64(species_seed)), Teff, logg, S, n_molecular=2,
                              metal_shift=feh, lam_ref_nm=lam_ref, D=D)
        wl = Workload("calibration_%s" % name, grid, atm, lines, zero_params(lines.L, S, xi))
        lam, sig = _atlas_pixels(grid, step, margin, R_atlas)
        for e in range(n_ep):
            w = telluric_weights(rng, lam, n_tell)
            out.append(CalStandard("%s_%d" % (name, e), wl, lam, sig, 3.0, (0.0, vb), w,
                                   1.0 / (len(CAL_STARS) * n_ep * float(np.sum(w)))))
    return out


def calibration(seed=240_006, n_records=CAL_RECORDS, n_bands=30):
    """The line-calibration workload of Sec. 6 on synthetic inputs: 1500-1700 nm
    at R = 300,000; 42,886 atomic records in complexes (18 species, neutral and
    singly ionised; calibrated) plus 18,000 molecular band lines (2 species;
    held fixed); a solar standard (5777 K, log g 4.44, xi 0.7 km/s, Gaussian
    dispersion 1.55 km/s) and an Arcturus-like giant (4286 K, log g 1.66,
    [M/H] -0.52, xi 1.7 km/s, 2.5 km/s) observed at two epochs.  Both stars
    share species properties (one species seed).  Atlas pixels every 1.5 (sun)
    and 1.4 (giant) native pixels with a Gaussian LSF of R = 250,000; telluric
    weights from 600 synthetic features per epoch; c gives each star equal
    total weight and its epochs equal shares, each a weighted mean square."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = 1500.0, 1700.0
    grid = grid_for(lo, hi, 3.0e5)
    atomic, cid = complex_lines(rng, n_records, lo, hi, 18)
    bands = band_lines(rng, n_bands, 600, lo, hi, [18, 19])
    lines = concat_lines(atomic, bands)
    active = np.arange(lines.L) < n_records
    std = _cal_standards(rng, grid, lines, 20, N_DEPTH, seed + 1, (1.5, 1.4), 2.5e5, 60, 600)
    return CalWorkload("1500-1700nm_R3e5_calibration_%d" % n_records, grid, lines, active, cid, std)


def calibration_tiny(seed=31, n_records=40, N=2500, D=24, lam_lo=1550.0):
    """A small calibration case with the same structure (n_records atomic records
    in complexes, a few band lines, the two stars, three spectra) on an
    N-pixel grid with D depths, for brute-force and oracle comparisons."""
    rng = np.random.Generator(np.random.PCG64(seed))
    grid = Grid(lam_lo, 3.0e5, N)
    hi = grid_last(grid)
    atomic, cid = complex_lines(rng, n_records, lam_lo + 0.2, hi - 0.2, 4)
    bands = band_lines(rng, 1, 6, lam_lo, hi, [4, 5])
    lines = concat_lines(atomic, bands)
    active = np.arange(lines.L) < n_records
    std = _cal_standards(rng, grid, lines, 6, D, seed + 1, (1.5, 1.4), 2.5e5, 60, 4)
    return CalWorkload("calibration_tiny_%d" % seed, grid, lines, active, cid, std)


def calibration_truth(rng, G):
    """Group corrections [4][G] drawn N(0, CAL_TRUTH_SIGMA) per row."""
    return np.stack([rng.normal(0.0, s, G) for s in CAL_TRUTH_SIGMA])
