"""CPU pins of the Limber oracle (``oracle/limber_approx.py``), Sec. 2.2 of arXiv:2410.03632.

* closed forms: Gaussian kernels and P = A k^-2 make every Limber integral a Gaussian
  moment (gg: zeroth, gs: second, ss: fourth), which pins N_t, f_t/k^2, the 1/chi^2 and
  the chi sum;
* the kernel derivatives of the extended approximation against analytic derivatives of
  K / sqrt(chi), with the convergence order of the 5-node stencil;
* the extended approximation against the same integral with analytic derivatives;
* the paper's claim that the extended approximation brings the gap to the exact
  (beyond-Limber) spectra from O(l^-2) to O(l^-4).
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import limber_approx as L


def _gauss(x, c, s):
    return np.exp(-0.5 * ((x - c) / s) ** 2)


def _moment(c1, s1, c2, s2, n):
    """int x^n g1 g2 dx for g = exp(-(x-c)^2 / 2 s^2): a Gaussian of mean mu and variance v."""
    v = 1.0 / (1.0 / s1 ** 2 + 1.0 / s2 ** 2)
    mu = v * (c1 / s1 ** 2 + c2 / s2 ** 2)
    amp = math.exp(-0.5 * (c1 - c2) ** 2 / (s1 ** 2 + s2 ** 2)) * math.sqrt(2 * math.pi * v)
    m = {0: 1.0, 2: mu ** 2 + v, 4: mu ** 4 + 6 * mu ** 2 * v + 3 * v ** 2}[n]
    return amp * m


def test_first_order_limber_gaussian_closed_forms():
    bins = [(1500.0, 120.0), (1800.0, 200.0)]   # one clustering, one shear bin
    chi, wchi = O.grid_chi(1601, 200.0, 3200.0)
    K = np.array([_gauss(chi, c, s) for c, s in bins])
    ell = np.array([10, 37, 200])
    A = 3.0e4
    P = A * L.limber_k(ell, chi) ** -2.0
    C = L.cl_limber(ell, chi, wchi, K, 1, 1, P)
    nu = ell + 0.5
    (c0, s0), (c1, s1) = bins
    Pi = (ell + 2.0) * (ell + 1.0) * ell * (ell - 1.0)
    # gg: (2/pi)(pi/2) int dchi/chi^2 K K A chi^2/nu^2
    ref_gg = A / nu ** 2 * _moment(c0, s0, c0, s0, 0)
    # gs: (2/pi) sqrt(Pi) (pi/2) int dchi/chi^2 K K (chi/nu)^2 A chi^2/nu^2
    ref_gs = np.sqrt(Pi) * A / nu ** 4 * _moment(c0, s0, c1, s1, 2)
    ref_ss = Pi * A / nu ** 6 * _moment(c1, s1, c1, s1, 4)
    for got, ref in zip(C, (ref_gg, ref_gs, ref_ss)):
        assert np.allclose(got, ref, rtol=1e-10, atol=0), (got / ref - 1)


def _kt_analytic(chi, c, s):
    """Kt = g / sqrt(chi), g = exp(-(chi-c)^2/2s^2): second and third derivatives by the
    product rule, with g' = -u g / s, g'' = (u^2 - 1) g / s^2, g''' = (3u - u^3) g / s^3,
    u = (chi - c)/s, and (chi^-1/2)^(n) = (-1/2)(-3/2)...(1/2 - n) chi^(-1/2 - n)."""
    u = (chi - c) / s
    g = np.exp(-0.5 * u ** 2)
    g1, g2, g3 = -u * g / s, (u ** 2 - 1) * g / s ** 2, (3 * u - u ** 3) * g / s ** 3
    h0 = chi ** -0.5
    h1, h2, h3 = -0.5 * chi ** -1.5, 0.75 * chi ** -2.5, -1.875 * chi ** -3.5
    d2 = g2 * h0 + 2 * g1 * h1 + g * h2
    d3 = g3 * h0 + 3 * g2 * h1 + 3 * g1 * h2 + g * h3
    return d2, d3


def test_kernel_derivatives_converge_at_the_stencil_order():
    c, s = 1500.0, 150.0
    errs = []
    for n in (201, 401, 801):
        chi = np.linspace(500.0, 2500.0, n)
        d2, d3 = L.kt_derivatives(chi, _gauss(chi, c, s))
        r2, r3 = _kt_analytic(chi, c, s)
        inner = slice(2, n - 2)
        errs.append((np.abs(d2[0, inner] - r2[inner]).max() / np.abs(r2).max(),
                     np.abs(d3[0, inner] - r3[inner]).max() / np.abs(r3).max()))
    (a2, a3), (b2, b3), (c2, c3) = errs
    assert a3 < 1e-2 and c3 < 1e-3 and c2 < 1e-5
    # centred 5-node stencil: second derivative O(h^4), third O(h^2)
    assert a2 / b2 > 12 and b2 / c2 > 12, errs
    assert a3 / b3 > 3.5 and b3 / c3 > 3.5, errs


def test_extended_limber_matches_analytic_derivatives():
    """The extended sums with stencil derivatives converge to the same sums with analytic
    derivatives at the order of the third-derivative stencil (O(h^2))."""
    bins = [(1500.0, 150.0), (1900.0, 250.0)]
    ell = np.array([5, 20, 80])
    nu = ell + 0.5
    errs = []
    for n in (2001, 4001):
        chi, wchi = O.grid_chi(n, 300.0, 3400.0)
        K = np.array([_gauss(chi, c, s) for c, s in bins])
        P = 2.0e4 * L.limber_k(ell, chi) ** -1.5
        C1 = L.cl_limber(ell, chi, wchi, K, 1, 1, P, order=1)
        C2 = L.cl_limber(ell, chi, wchi, K, 1, 1, P, order=2)
        A = []
        for c, s in bins:
            d2, d3 = _kt_analytic(chi, c, s)
            A.append(np.sqrt(chi) * (0.5 * chi ** 2 * d2 + chi ** 3 / 6 * d3))
        k = L.limber_k(ell, chi)
        err = 0.0
        for p, (t, i, j) in enumerate(L.pairs(1, 1)):
            kk = K[i] * K[j] - (A[i] * K[j] + K[i] * A[j])[None, :] / nu[:, None] ** 2
            g = {"gg": 1.0, "gs": k ** -2.0, "ss": k ** -4.0}[t]
            ref = L.prefactor(t, ell) * 0.5 * math.pi * (wchi * kk * g * P / chi ** 2).sum(axis=1)
            # error relative to the size of the correction itself
            err = max(err, np.abs((C2[p] - ref) / (ref - C1[p])).max())
            assert abs(C2[p][0] / C1[p][0] - 1) > 1e-3      # the correction matters at low ell
        errs.append(err)
    assert errs[1] < 2e-3 and 3.5 < errs[0] / errs[1] < 4.5, errs


def _graded(n, a, b):
    """n Gauss-Legendre nodes on [a, b], graded towards b (s -> 1 - (1-s)^3)."""
    x, w = np.polynomial.legendre.leggauss(n)
    s = 0.5 * (x + 1)
    t = 1 - (1 - s) ** 3
    return a + (b - a) * t, 0.5 * w * 3 * (1 - s) ** 2 * (b - a)


def test_extended_limber_gap_falls_faster_than_first_order():
    """Sec. 2.2: the extended approximation brings the error from O(l^-2) to O(l^-4).
    Exact spectra from the oracle's continuous chi-R integral with a pure power law.  This
    also fixes the sign of the correction bracket: with the printed plus sign the gap grows
    (it roughly doubles the first-order gap) and keeps falling like l^-2."""
    ell = [25, 50, 100]
    kmin, kmax, N = 1e-4, 1.0, 64
    k, _ = O.grid_k(N, kmin, kmax)
    nodal = k ** -2.0
    lo, hi = 900.0, 2300.0
    types = "gg gs ss".split()
    K = lambda xx: np.array([_gauss(xx, 1600.0, 150.0)] * 2)
    xg, wg = np.polynomial.legendre.leggauss(56)
    chi = lo + (hi - lo) * 0.5 * (xg + 1)
    wchi = 0.5 * (hi - lo) * wg
    R, wR = _graded(96, 0.4, 1.0)
    c1 = np.repeat(chi, len(R))
    c2 = (chi[:, None] * R[None, :]).ravel()
    w = O.w_points(ell, types, kmin, kmax, c1, c2, nc=N, P=nodal, shared=True)
    C_ex = O.sum_rform(chi, wchi, wR, 1, 1, K(chi), K(c2).reshape(2, len(chi), len(R)), ell, types, w)
    P = L.limber_k(ell, chi) ** -2.0
    gap1 = np.abs(L.cl_limber(ell, chi, wchi, K(chi), 1, 1, P, order=1) / C_ex - 1)
    gap2 = np.abs(L.cl_limber(ell, chi, wchi, K(chi), 1, 1, P, order=2) / C_ex - 1)
    print("first-order gaps", gap1, "\nextended gaps", gap2)
    for p in range(3):
        assert np.all(gap2[p] < gap1[p]), (types[p], gap1[p], gap2[p])
        assert np.all(gap2[p, 1:] < 0.2 * gap1[p, 1:]), (types[p], gap1[p], gap2[p])
        # falls by much more than the first-order factor ~4 per doubling of ell (at l = 100 the
        # gap is at the 3e-4..5e-4 accuracy of the exact spectra)
        assert gap2[p, 0] / gap2[p, 1] > 7.0, (types[p], gap2[p])
        assert gap2[p, 2] < 1e-3


def test_nonlinear_correction_is_the_limber_sum_of_the_difference():
    chi, wchi = O.grid_chi(64, 200.0, 3000.0)
    rng = np.random.default_rng(0)
    K = rng.random((3, 64))
    ell = np.array([2, 30, 300])
    Plin = rng.random((3, 64)) + 1.0
    Pnl = Plin * (1 + rng.random((3, 64)))
    for order in (1, 2):
        d = L.cl_limber(ell, chi, wchi, K, 2, 1, Pnl, P_sub=Plin, order=order)
        ref = L.cl_limber(ell, chi, wchi, K, 2, 1, Pnl, order=order) - \
            L.cl_limber(ell, chi, wchi, K, 2, 1, Plin, order=order)
        assert np.allclose(d, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())
        assert np.array_equal(L.cl_limber(ell, chi, wchi, K, 2, 1, Plin, P_sub=Plin, order=order),
                              np.zeros_like(d))
