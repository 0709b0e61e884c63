"""Limber approximations of the angular spectra (FP64, numpy): TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import this module; it shares nothing with the HIP library.

Sec. 2.2 of arXiv:2410.03632 ("The Limber approximation"): replacing the two Bessel
functions by their peak, k chi = l + 1/2, turns the k-integral into
    int dk f_t(k) P(k) j_l(k chi1) j_l(k chi2) -> (pi / 2 chi^2) [f_t P / k^2]_{k = nu/chi} delta(chi1 - chi2),
nu = l + 1/2 (the closure relation of the Bessel functions, normalised as
int dk k^2 j_l(k x) j_l(k y) = pi/(2 x^2) delta(x - y)), so with the prefactors N_t(l) of
Eqs. gg, gs, ss the spectrum of the bin pair (i, j) of type t is
    C^limb_ij(l) = N_t(l) (pi/2) int dchi/chi^2 K_i(chi) K_j(chi) f_t(k)/k^2 P(k, chi, chi),  k = nu/chi,
and for gg (N = 2/pi, f = k^2) this is the paper's first-order Limber integral.

The extended (second-order) Limber approximation of the same section (after LoVerde &
Afshordi 2008) multiplies the integrand by
    1 - nu^-2 [ chi^2/2 (Kt_i''/Kt_i + Kt_j''/Kt_j) + chi^3/6 (Kt_i'''/Kt_i + Kt_j'''/Kt_j) ],
Kt = K / sqrt(chi).  The paper prints the bracket with a plus sign; with that sign the
approximation moves away from the exact spectra and its error stays O(nu^-2), against the
O(nu^-4) the same section states, while the minus sign of the expansion of the Bessel
integral gives the stated order (checked against the oracle's exact spectra).  Since
K_i K_j Kt_i''/Kt_i = sqrt(chi) Kt_i'' K_j, the oracle evaluates
    K_i K_j - nu^-2 sqrt(chi) [ (chi^2/2 Kt_i'' + chi^3/6 Kt_i''') K_j + K_i (chi^2/2 Kt_j'' + chi^3/6 Kt_j''') ],
which is the same expression without the division (kernels may vanish).  For the gs and
ss types the expansion is applied with f_t P / k^2 in place of P (the Bessel expansion
acts on the kernels only).

The discrete definition (the parity target of the GPU path):
  * the chi integral is the plan's quadrature sum_a wchi_a (...)(chi_a);
  * P is supplied by the caller at the Limber points (k = nu/chi_a, chi_a): P[l][a];
  * Kt'' and Kt''' at node a are the derivatives at chi_a of the degree-4 polynomial
    through (chi_s, Kt(chi_s)) for the 5 nodes s = a-2..a+2, shifted to the first / last
    five nodes at the two ends of the grid (here: an exact fit by numpy.polyfit in the
    local variable chi - chi_a, differentiated exactly).
The non-linear correction of Sec. 3.2 is C_tot = C_lin + C^limb[P_nl] - C^limb[P_lin], i.e.
the Limber sum of the difference of the two spectra added to the beyond-Limber C_lin.
"""
from __future__ import annotations

import math

import numpy as np

TYPES = ("gg", "gs", "ss")


def prefactor(t: str, ell) -> np.ndarray:
    """N_t(l) of Eqs. gg, gs, ss: 2/pi, (2/pi) sqrt(Pi_l), (2/pi) Pi_l, Pi_l = (l+2)(l+1)l(l-1)."""
    l = np.asarray(ell, dtype=np.float64)
    Pi = (l + 2) * (l + 1) * l * (l - 1)
    return {"gg": 2 / math.pi * np.ones_like(l), "gs": 2 / math.pi * np.sqrt(Pi), "ss": 2 / math.pi * Pi}[t]


def pairs(n_g: int, n_s: int, types=TYPES):
    out = []
    if "gg" in types:
        out += [("gg", i, j) for i in range(n_g) for j in range(i, n_g)]
    if "gs" in types:
        out += [("gs", i, n_g + j) for i in range(n_g) for j in range(n_s)]
    if "ss" in types:
        out += [("ss", n_g + i, n_g + j) for i in range(n_s) for j in range(i, n_s)]
    return out


def limber_k(ell, chi) -> np.ndarray:
    """Limber points k[l][a] = (l + 1/2) / chi_a."""
    return (np.asarray(ell, dtype=np.float64)[:, None] + 0.5) / np.asarray(chi, dtype=np.float64)[None, :]


def kt_derivatives(chi, K):
    """(Kt'', Kt''') at every node for Kt = K / sqrt(chi): exact derivatives of the degree-4
    interpolant through the 5 nearest nodes (end nodes use the first / last five)."""
    chi = np.asarray(chi, dtype=np.float64)
    K = np.atleast_2d(np.asarray(K, dtype=np.float64))
    n = chi.size
    if n < 5:
        raise ValueError("the extended Limber approximation needs at least 5 chi nodes")
    Kt = K / np.sqrt(chi)[None, :]
    d2 = np.empty_like(Kt)
    d3 = np.empty_like(Kt)
    for a in range(n):
        s0 = min(max(a - 2, 0), n - 5)
        x = chi[s0:s0 + 5] - chi[a]
        for b in range(K.shape[0]):
            c = np.polyfit(x, Kt[b, s0:s0 + 5], 4)     # highest degree first
            # derivatives at x = 0: p'' = 2 c[2], p''' = 6 c[1]
            d2[b, a] = 2.0 * c[2]
            d3[b, a] = 6.0 * c[1]
    return d2, d3


def cl_limber(ell, chi, wchi, K, n_g, n_s, P, *, P_sub=None, order=1, types=TYPES):
    """C^limb[p][l] for the pairs of (n_g, n_s) in the output order (gg, gs, ss).

    ell [n_l]; chi, wchi [n_chi]; K [bins][n_chi] (the calligraphic kernels at chi_a);
    P [n_l][n_chi] = P(k = (l+1/2)/chi_a, chi_a, chi_a); P_sub, if given, is subtracted
    (non-linear minus linear spectrum); order 1 (Limber) or 2 (extended Limber)."""
    ell = np.asarray(ell, dtype=np.float64)
    chi = np.asarray(chi, dtype=np.float64)
    wchi = np.asarray(wchi, dtype=np.float64)
    K = np.asarray(K, dtype=np.float64)
    dP = np.asarray(P, dtype=np.float64) - (0.0 if P_sub is None else np.asarray(P_sub, dtype=np.float64))
    nu = ell + 0.5
    k = limber_k(ell, chi)
    if order == 2:
        d2, d3 = kt_derivatives(chi, K)
        A = np.sqrt(chi)[None, :] * (0.5 * chi ** 2 * d2 + chi ** 3 / 6.0 * d3)   # [bins][n_chi]
    out = []
    for t, i, j in pairs(n_g, n_s, types):
        kk = K[i] * K[j]                                           # [n_chi]
        if order == 2:
            corr = (A[i] * K[j] + K[i] * A[j])[None, :] / nu[:, None] ** 2
            kk = kk[None, :] - corr
        else:
            kk = np.broadcast_to(kk, k.shape)
        g = {"gg": np.ones_like(k), "gs": 1.0 / k ** 2, "ss": 1.0 / k ** 4}[t]   # f_t / k^2
        s = (wchi[None, :] * kk * g * dP / chi[None, :] ** 2).sum(axis=1)
        out.append(prefactor(t, ell) * 0.5 * math.pi * s)
    return np.array(out)
