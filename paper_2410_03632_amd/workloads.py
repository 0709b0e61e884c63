"""Seeded synthetic 3x2pt inputs: multipole lists, tomographic kernels and P(k, chi1, chi2).

This module holds input generation only, none of the C_ell method's arithmetic: it
evaluates a synthetic power spectrum and tomographic window functions at points
that the caller supplies (the k nodes and the (chi, R*chi) evaluation points of a
plan).  Both the CPU oracle and the HIP path consume what it produces.

Physics of the inputs (paper Sec. "The Blast algorithm", Eqs. gg/ss/gs and the
kernel definitions that follow them):

* clustering window  W^g(chi) = n(chi)  (unit linear bias, n normalised in chi);
* lensing window     W^s(chi) = 3/2 Omega_m (H0/c)^2 chi/a(chi)
                                 * int_chi^inf dchi' n(chi') (chi'-chi)/chi'
  for a flat LCDM background (Omega_m = 0.3, h = 0.7);
* the kernels handed to the C_ell evaluation are the paper's calligraphic K
  (Eq. final_cls): K = W for clustering and K = W / chi^2 for lensing;
* P(k, chi1, chi2) = A k^ns / (1 + (k/0.02)^2.8) (1 + 0.05 sin(150 k) e^{-(k/0.2)^2})
                     * D(chi1) D(chi2),   D(chi) = 1 / (1 + chi/Ds).
  The paper allows an unequal-time P with general c_n(chi1, chi2); the separable
  product above is one such spectrum and is symmetric in chi1 <-> chi2.

Random draws use numpy's PCG64 with seed = 2410_03632 + 1000*config + index, in the
order A, tilt, D-scale, bins, ell subset, arrival gap.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 2410_03632
C_KMS = 299_792.458          # speed of light [km/s]
H0 = 70.0                    # [km/s/Mpc], h = 0.7
OMEGA_M = 0.3

# ----------------------------------------------------------------------------
# multipoles
# ----------------------------------------------------------------------------


def ell_list(n: int, lmin: int, lmax: int) -> np.ndarray:
    """n integer multipoles, log-spaced on [lmin, lmax], strictly increasing.

    round(geomspace) and then every duplicate is bumped to previous + 1 (the default
    workloads use integer ell; real_ell_list gives the challenge's kind of list)."""
    raw = np.rint(np.geomspace(lmin, lmax, n)).astype(np.int64)
    out = raw.copy()
    for i in range(1, n):
        if out[i] <= out[i - 1]:
            out[i] = out[i - 1] + 1
    if out[-1] > lmax:
        raise ValueError("cannot fit %d distinct integer ells in [%d, %d]" % (n, lmin, lmax))
    return out.astype(np.int32)


def real_ell_list(n: int, lmin: float, lmax: float) -> np.ndarray:
    """n log-spaced multipoles on [lmin, lmax], not rounded: the kind of multipole list the
    paper's challenge evaluates (its values are not integers)."""
    return np.geomspace(lmin, lmax, n)


# ----------------------------------------------------------------------------
# configurations (grid shapes and tomographic layouts)
# ----------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    n_ell: int
    ell_min: int
    ell_max: int
    n_chi: int
    chi_min: float
    chi_max: float
    n_R: int
    R_min: float
    n_cheb: int
    k_min: float
    k_max: float
    g_centres: tuple
    g_sigma: float
    s_centres: tuple
    s_sigma: float

    @property
    def n_g(self) -> int:
        return len(self.g_centres)

    @property
    def n_s(self) -> int:
        return len(self.s_centres)

    def ells(self) -> np.ndarray:
        return ell_list(self.n_ell, self.ell_min, self.ell_max)


CONFIGS = {
    # small: 2 clustering + 2 lensing bins from the same two Gaussian n(chi)
    1: Config("small", 20, 2, 200, 64, 50.0, 3000.0, 32, 0.3, 64, 1e-4, 10.0,
              (800.0, 1600.0), 150.0, (800.0, 1600.0), 150.0),
    # full 3x2pt: 10 clustering bins + 5 broad source bins (120 pairs)
    2: Config("full3x2pt", 96, 2, 1000, 256, 20.0, 4500.0, 96, 0.3, 128, 1e-4, 10.0,
              tuple(500.0 + 300.0 * i for i in range(10)), 150.0,
              tuple(1200.0 + 600.0 * i for i in range(5)), 400.0),
}


def tiny_config(n_ell=6, ell_max=40, n_chi=12, n_R=10, n_cheb=24, k_max=0.6,
                chi_min=300.0, chi_max=1500.0, n_g=2, n_s=2) -> Config:
    """A small configuration the oracle finishes in seconds (parity tests)."""
    gc = tuple(np.linspace(chi_min + 0.3 * (chi_max - chi_min),
                           chi_min + 0.7 * (chi_max - chi_min), n_g))
    sc = tuple(np.linspace(chi_min + 0.4 * (chi_max - chi_min),
                           chi_min + 0.8 * (chi_max - chi_min), n_s))
    return Config("tiny", n_ell, 2, ell_max, n_chi, chi_min, chi_max, n_R, 0.3, n_cheb,
                  1e-4, k_max, gc, 0.12 * (chi_max - chi_min), sc, 0.2 * (chi_max - chi_min))


def seed_for(config: int, index: int = 0) -> int:
    return SEED_BASE + 1000 * config + index


# ----------------------------------------------------------------------------
# background cosmology (input physics only)
# ----------------------------------------------------------------------------

_ZTAB = None


def _z_of_chi_table():
    global _ZTAB
    if _ZTAB is None:
        z = np.linspace(0.0, 20.0, 200_001)
        ez = np.sqrt(OMEGA_M * (1 + z) ** 3 + 1 - OMEGA_M)
        integrand = 1.0 / ez
        chi = np.concatenate([[0.0], np.cumsum(0.5 * (integrand[1:] + integrand[:-1]) * np.diff(z))])
        chi *= C_KMS / H0
        _ZTAB = (chi, z)
    return _ZTAB


def z_of_chi(chi):
    tab_chi, tab_z = _z_of_chi_table()
    return np.interp(np.asarray(chi, dtype=np.float64), tab_chi, tab_z)


# ----------------------------------------------------------------------------
# tomographic kernels
# ----------------------------------------------------------------------------


def nz_gauss(chi, centre, sigma):
    """Gaussian n(chi), normalised so that int_0^inf n dchi = 1."""
    chi = np.asarray(chi, dtype=np.float64)
    norm = 0.5 * math.erfc(-centre / (math.sqrt(2.0) * sigma)) * math.sqrt(2 * math.pi) * sigma
    return np.exp(-0.5 * ((chi - centre) / sigma) ** 2) / norm


def lensing_window(chi, centre, sigma, n_fine=40_001):
    """W^s(chi) for a Gaussian source n(chi) (flat LCDM), evaluated at chi >= 0."""
    chi = np.asarray(chi, dtype=np.float64)
    top = centre + 12.0 * sigma
    grid = np.linspace(0.0, top, n_fine)
    n = nz_gauss(grid, centre, sigma)
    with np.errstate(divide="ignore"):
        n_over = np.where(grid > 0, n / np.maximum(grid, 1e-300), 0.0)
    # F0(x) = int_x^top n, F1(x) = int_x^top n / chi'   (trapezoid, accumulated from the top)
    def tail(f):
        seg = 0.5 * (f[1:] + f[:-1]) * np.diff(grid)
        return np.concatenate([np.cumsum(seg[::-1])[::-1], [0.0]])
    F0 = tail(n)
    F1 = tail(n_over)
    f0 = np.interp(chi, grid, F0, right=0.0)
    f1 = np.interp(chi, grid, F1, right=0.0)
    pref = 1.5 * OMEGA_M * (H0 / C_KMS) ** 2
    a_inv = 1.0 + z_of_chi(chi)
    w = pref * chi * a_inv * (f0 - chi * f1)
    return np.maximum(w, 0.0)


def calK(chi, kind, centre, sigma):
    """The calligraphic kernel of Eq. final_cls: W for clustering, W/chi^2 for lensing."""
    chi = np.asarray(chi, dtype=np.float64)
    if kind == "g":
        return nz_gauss(chi, centre, sigma)
    w = lensing_window(chi, centre, sigma)
    return w / (chi * chi)


def kernels(cfg_bins, chi, chi2):
    """Kernel tables for every bin.

    cfg_bins : list of (kind, centre, sigma), clustering bins first.
    chi      : [n_chi] evaluation points chi_a.
    chi2     : [n_chi, n_R] evaluation points R_b chi_a.
    Returns Kchi [n_bins, n_chi] and Kchi2 [n_bins, n_chi, n_R] (float64)."""
    nb = len(cfg_bins)
    Kchi = np.empty((nb, len(chi)))
    Kchi2 = np.empty((nb,) + tuple(np.shape(chi2)))
    for i, (kind, c, s) in enumerate(cfg_bins):
        Kchi[i] = calK(chi, kind, c, s)
        Kchi2[i] = calK(np.ravel(chi2), kind, c, s).reshape(np.shape(chi2))
    return Kchi, Kchi2


def bins_of(cfg: Config):
    return [("g", c, cfg.g_sigma) for c in cfg.g_centres] + [("s", c, cfg.s_sigma) for c in cfg.s_centres]


# ----------------------------------------------------------------------------
# synthetic power spectrum
# ----------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class Cosmo:
    A: float
    ns: float = 0.96
    Ds: float = 4000.0


def draw_cosmo(rng: np.random.Generator, vary: bool = False) -> Cosmo:
    A = float(rng.uniform(1e4, 3e4))
    if not vary:
        return Cosmo(A)
    ns = float(rng.uniform(0.9, 1.0))
    Ds = float(rng.uniform(3000.0, 5000.0))
    return Cosmo(A, ns, Ds)


def p0(k, cosmo: Cosmo):
    k = np.asarray(k, dtype=np.float64)
    base = cosmo.A * k ** cosmo.ns / (1.0 + (k / 0.02) ** 2.8)
    return base * (1.0 + 0.05 * np.sin(150.0 * k) * np.exp(-(k / 0.2) ** 2))


def growth(chi, cosmo: Cosmo):
    return 1.0 / (1.0 + np.asarray(chi, dtype=np.float64) / cosmo.Ds)


def p_grid(k, chi, chi2, cosmo: Cosmo):
    """P(k_j, chi_a, R_b chi_a) as [n_chi, n_R, n_k] float64 (k fastest)."""
    pk = p0(k, cosmo)
    d1 = growth(chi, cosmo)[:, None]
    d2 = growth(chi2, cosmo)
    return (d1 * d2)[:, :, None] * pk[None, None, :]


# ----------------------------------------------------------------------------
# one full synthetic input set
# ----------------------------------------------------------------------------


@dataclasses.dataclass
class Inputs:
    cosmo: Cosmo
    P: np.ndarray        # [n_chi, n_R, n_cheb]
    Kchi: np.ndarray     # [n_bins, n_chi]
    Kchi2: np.ndarray    # [n_bins, n_chi, n_R]
    n_g: int
    n_s: int


def make_inputs(cfg: Config, seed: int, k_nodes, chi, R, vary=False) -> Inputs:
    """Draw a cosmology with `seed` and evaluate P and the kernels at the plan's
    points: k nodes (ascending), chi nodes and R nodes (chi2 = R_b chi_a)."""
    rng = np.random.default_rng(seed)
    cosmo = draw_cosmo(rng, vary)
    chi = np.asarray(chi, dtype=np.float64)
    chi2 = chi[:, None] * np.asarray(R, dtype=np.float64)[None, :]
    P = p_grid(k_nodes, chi, chi2, cosmo)
    Kchi, Kchi2 = kernels(bins_of(cfg), chi, chi2)
    return Inputs(cosmo, P, Kchi, Kchi2, cfg.n_g, cfg.n_s)


def pair_list(n_g: int, n_s: int, types=("gg", "gs", "ss")):
    """Bin-pair order of the output: gg (i<=j), then gs (i over g, j over s),
    then ss (i<=j).  Bin indices are global (clustering first)."""
    out = []
    if "gg" in types:
        out += [("gg", i, j) for i in range(n_g) for j in range(i, n_g)]
    if "gs" in types:
        out += [("gs", i, n_g + j) for i in range(n_g) for j in range(n_s)]
    if "ss" in types:
        out += [("ss", n_g + i, n_g + j) for i in range(n_s) for j in range(i, n_s)]
    return out


# ----------------------------------------------------------------------------
# serving workload: Poisson stream of requests with uneven bins and multipoles
# ----------------------------------------------------------------------------

SERVING = Config("serving", 200, 2, 1000, 256, 20.0, 4500.0, 96, 0.3, 128, 1e-4, 10.0,
                 tuple(500.0 + 280.0 * i for i in range(15)), 150.0,
                 tuple(1200.0 + 600.0 * i for i in range(5)), 400.0)


@dataclasses.dataclass
class ServingRequest:
    cosmo: Cosmo
    n_g: int
    n_s: int
    ell_idx: np.ndarray   # increasing indices into the 200-multipole master list
    gap_s: float          # time since the previous arrival


def serving_requests(n: int, rate_hz: float = 200.0, index0: int = 0):
    """n requests of the serving configuration: each draws (in this order) a cosmology
    (A, tilt, D-scale), its bins (3-15 clustering, 1-5 shear), a sorted subset of 20-200 of
    the master multipoles and an exponential arrival gap of mean 1/rate."""
    out = []
    for i in range(n):
        rng = np.random.default_rng(seed_for(4, index0 + i))
        cos = draw_cosmo(rng, vary=True)
        ng = int(rng.integers(3, 16))
        ns = int(rng.integers(1, 6))
        nl = int(rng.integers(20, 201))
        idx = np.sort(rng.choice(SERVING.n_ell, size=nl, replace=False)).astype(np.int32)
        gap = float(rng.exponential(1.0 / rate_hz))
        out.append(ServingRequest(cos, ng, ns, idx, gap))
    return out


def request_kernels(Kchi, Kchi2, n_g, n_s, max_g=15):
    """Kernel tables of a request that uses the first n_g clustering and n_s shear bins of
    the serving layout (tables for all 15 + 5 bins given)."""
    sel = list(range(n_g)) + [max_g + j for j in range(n_s)]
    return np.ascontiguousarray(Kchi[sel]), np.ascontiguousarray(Kchi2[sel])


# ----------------------------------------------------------------------------
# differentiable kernels (torch): the same windows as functions of the Gaussian
# centres and widths, smooth in those parameters so that gradients through them
# can be checked by finite differences
# ----------------------------------------------------------------------------

_GL16 = np.polynomial.legendre.leggauss(16)


def _unit_rule(panels: int):
    """Composite 16-point Gauss-Legendre nodes and weights on [0, 1]."""
    x, w = _GL16
    s = (np.arange(panels)[:, None] + 0.5 * (x[None, :] + 1.0)) / panels
    return s.ravel(), np.repeat(np.full(panels, 0.5 / panels), 16) * np.tile(w, panels)


def kernels_torch(kinds, centres, sigmas, chi, chi2, panels: int = 32):
    """Kernel tables K_chi [n_bins, n_chi] and K_chi2 [n_bins, n_chi, n_R] (torch float64,
    on the device of `centres`) for Gaussian bins, differentiable in `centres` and `sigmas`.

    kinds : sequence of "g" / "s" (clustering bins first, as in `kernels`).
    The clustering kernel is n(chi) as in `nz_gauss`.  The lensing kernel W^s/chi^2 uses
    the substitution chi' = chi e^u in the efficiency integral,
        int_chi^inf n(chi') (chi' - chi)/chi' dchi' = chi int_0^U n(chi e^u) (e^u - 1) du,
    with U = ln(max(c + 12 sigma, chi)/chi), on composite Gauss-Legendre nodes in u; the
    integrand and U are smooth in (c, sigma).  It agrees with `lensing_window` to its
    trapezoid error (about 1e-7 relative)."""
    import torch

    dev = centres.device
    dt = torch.float64
    pts = np.concatenate([np.ravel(chi), np.ravel(chi2)])
    x = torch.as_tensor(pts, dtype=dt, device=dev)
    a_inv = torch.as_tensor(1.0 + z_of_chi(pts), dtype=dt, device=dev)
    s_nodes, s_w = (torch.as_tensor(v, dtype=dt, device=dev) for v in _unit_rule(panels))
    pref = 1.5 * OMEGA_M * (H0 / C_KMS) ** 2
    out = []
    for i, kind in enumerate(kinds):
        c, sg = centres[i], sigmas[i]
        norm = 0.5 * torch.special.erfc(-c / (math.sqrt(2.0) * sg)) * math.sqrt(2.0 * math.pi) * sg

        def n_of(y):
            return torch.exp(-0.5 * ((y - c) / sg) ** 2) / norm

        if kind == "g":
            out.append(n_of(x))
            continue
        top = c + 12.0 * sg
        U = torch.log(torch.clamp(top / x, min=1.0))                     # [P]
        u = U[:, None] * s_nodes[None, :]                                  # [P, Q]
        eff = (n_of(x[:, None] * torch.exp(u)) * torch.expm1(u) * s_w[None, :]).sum(dim=1) * U
        out.append(pref * a_inv * eff)                                     # W^s / chi^2
    K = torch.stack(out)
    n_chi = np.size(chi)
    return K[:, :n_chi].contiguous(), K[:, n_chi:].reshape((len(kinds),) + tuple(np.shape(chi2))).contiguous()


# ----------------------------------------------------------------------------
# spectra at the Limber points (k = (l+1/2)/chi, chi1 = chi2 = chi) and a non-linear stand-in
# ----------------------------------------------------------------------------


def nl_boost(k, chi):
    """Synthetic non-linear boost P_nl / P_lin = 1 + (k / k_nl(chi))^1.5 with k_nl = 0.2 (1 + chi/2000)
    [1/Mpc]: smooth, larger at small scales and late times; a stand-in, not a fit."""
    k = np.asarray(k, dtype=np.float64)
    knl = 0.2 * (1.0 + np.asarray(chi, dtype=np.float64) / 2000.0)
    return 1.0 + (k / knl) ** 1.5


def p_limber(k_limb, chi, cosmo: Cosmo, nonlinear: bool = False):
    """P(k[l][a], chi_a, chi_a) on the Limber points k_limb [n_ell, n_chi] (linear, or with the
    synthetic non-linear boost)."""
    chi = np.asarray(chi, dtype=np.float64)
    P = p0(k_limb, cosmo) * growth(chi, cosmo)[None, :] ** 2
    return P * nl_boost(k_limb, chi[None, :]) if nonlinear else P
