"""Pins of the CPU oracle against facts fixed by mathematics and by the paper.

Each test checks one ingredient of the oracle against something other than the
oracle itself: arbitrary-precision Bessel values (mpmath), a library quadrature
rule, exactness of quadrature on polynomials, the Chebyshev interpolation and
aliasing identities (Eqs. chebpoints, a2, cheb2), Weber's closed form for a
Gaussian spectrum, the chi1-chi2 form of Eq. cls-general against the chi-R form
of Eq. final_cls, and the approach to the Limber limit at high multipole.
"""
import math

import mpmath as mp
import numpy as np
import pytest
import scipy.special as sp

import oracle as O
from paper_2410_03632_amd import workloads as W

mp.mp.dps = 40


def j_mp(l, x):
    x = mp.mpf(x)
    return float(mp.sqrt(mp.pi / (2 * x)) * mp.besselj(l + mp.mpf(1) / 2, x))


# ----------------------------------------------------------------------------- Bessel

@pytest.mark.parametrize("x", [1e-7, 1e-3, 0.3, 0.999, 1.0, 3.7, 42.0, 199.5, 500.0, 999.9, 1000.5, 4.3e4])
def test_bessel_vs_mpmath(x):
    lmax = 1000
    j = O.sph_jn(lmax, x)
    for l in [0, 1, 2, 3, 7, 20, 64, 150, 199, 200, 201, 450, 499, 500, 501, 700, 999, 1000]:
        ref = j_mp(l, x)
        if abs(ref) < 1e-280:
            assert abs(j[l]) < 1e-270
            continue
        # oscillatory region: error relative to the local envelope ~ 1/x; decaying region: relative
        env = abs(ref) if l > x else max(abs(ref), 1.0 / x)
        assert abs(j[l] - ref) <= 2e-12 * env, (l, x, j[l], ref)


@pytest.mark.parametrize("x", [0.05, 2.0, 77.7, 640.0, 2500.0])
def test_bessel_vs_scipy_whole_array(x):
    lmax = 800
    j = O.sph_jn(lmax, x)
    ref = sp.spherical_jn(np.arange(lmax + 1), x)
    ls = np.arange(lmax + 1)
    env = np.where(ls > x, np.abs(ref), np.maximum(np.abs(ref), 1.0 / x))
    m = np.abs(ref) > 1e-250
    assert np.all(np.abs(j[m] - ref[m]) <= 1e-10 * env[m])


def test_bessel_small_x_series_and_large_x_asymptote():
    # j_l(x) = x^l/(2l+1)!! (1 - x^2/(2(2l+3)) + ...) for x -> 0
    x = 1e-4
    j = O.sph_jn(12, x)
    for l in range(13):
        dfact = float(np.prod(np.arange(2 * l + 1, 0, -2, dtype=np.float64)))
        ser = x ** l / dfact * (1 - x * x / (2 * (2 * l + 3)))
        assert abs(j[l] / ser - 1) < 1e-12
    # j_l(x) -> sin(x - l pi/2)/x for x >> l^2
    x = 2.0e6 + 0.3
    j = O.sph_jn(5, x)
    for l in range(6):
        assert abs(j[l] - math.sin(x - l * math.pi / 2) / x) < 1e-5 / x


def test_bessel_branch_continuity():
    # the upward / downward switch happens at x = lmax; both sides must agree smoothly
    lmax = 300
    for x in [lmax - 1e-9, lmax + 1e-9]:
        j = O.sph_jn(lmax, x)
        for l in [0, 100, 299, 300]:
            assert abs(j[l] - j_mp(l, x)) < 1e-12 * max(abs(j_mp(l, x)), 1.0 / x)


# ----------------------------------------------------------------------------- quadrature rules

@pytest.mark.parametrize("x", [1e-4, 0.37, 2.0, 29.5, 30.5, 111.1, 640.0, 1200.0])
def test_real_order_bessel_vs_mpmath(x):
    """Non-integer multipoles: j_nu(x) = sqrt(pi/2x) J_{nu+1/2}(x) for real nu (mpmath, 40 digits)."""
    for nu in [0.0, 0.25, 0.5, 0.999, 1.5, 2.37, 10.5, 57.75, 211.63, 640.2, 999.5, 1500.01]:
        xm = mp.mpf(x)
        ref = float(mp.sqrt(mp.pi / (2 * xm)) * mp.besselj(mp.mpf(nu) + mp.mpf(1) / 2, xm))
        got = O.sph_jnu(nu, x)
        if abs(ref) < 1e-280:
            assert abs(got) < 1e-270
            continue
        env = abs(ref) if nu > x else max(abs(ref), 1.0 / x)
        assert abs(got - ref) <= 1e-12 * env, (nu, x, got, ref)


@pytest.mark.parametrize("x", [0.05, 3.0, 77.7, 640.0, 2500.0])
def test_real_order_bessel_at_integer_orders_equals_integer_recurrence(x):
    """The fractional-order routine (one sequence per order, Neumann normalisation) and the
    integer routine (one sequence for all orders, closed-form j_0 / j_1 normalisation) are
    different computations that must agree at integer orders."""
    lmax = 800
    j = O.sph_jn(lmax, x)
    for l in [0, 1, 2, 5, 33, 200, 799]:
        got = O.sph_jnu(float(l), x)
        env = abs(j[l]) if l > x else max(abs(j[l]), 1.0 / x)
        if abs(j[l]) < 1e-250:
            continue
        assert abs(got - j[l]) <= 1e-12 * env, (l, x, got, j[l])


def test_real_order_bessel_recurrence_in_order():
    """j_{nu-1} + j_{nu+1} = (2 nu + 1)/x j_nu for fractional nu (catches an offset of the
    fractional part or of the cylindrical order)."""
    for x in [0.8, 9.0, 45.0, 300.0]:
        for nu in [1.3, 4.61, 25.5, 120.05]:
            a, b, c = O.sph_jnu(nu - 1, x), O.sph_jnu(nu, x), O.sph_jnu(nu + 1, x)
            scale = max(abs(a), abs(c), abs(b) * (2 * nu + 1) / x, 1e-300)
            assert abs(a + c - (2 * nu + 1) / x * b) <= 1e-12 * scale, (x, nu)


def test_real_prefactors_against_gamma():
    """N_t(l) for non-integer l: (l+2)!/(l-2)! continues as Gamma(l+3)/Gamma(l-1)."""
    for l in [2.0, 2.5, 17.3, 211.63, 999.9]:
        r = math.exp(math.lgamma(l + 3) - math.lgamma(l - 1))
        assert abs(O.prefactor("gg", l) - 2 / math.pi) < 1e-16
        assert abs(O.prefactor("gs", l) / (2 / math.pi * math.sqrt(r)) - 1) < 1e-12
        assert abs(O.prefactor("ss", l) / (2 / math.pi * r) - 1) < 1e-12


def test_gl16_matches_library():
    x, w = O.gl16()
    xr, wr = np.polynomial.legendre.leggauss(16)
    o = np.argsort(x)
    assert np.allclose(x[o], xr, atol=1e-15, rtol=0)
    assert np.allclose(w[o], wr, atol=1e-15, rtol=0)


@pytest.mark.parametrize("n", [4, 5, 9, 64, 96, 256])
def test_simpson_even_exact_on_cubics(n):
    lo, hi = 26.0, 7000.0
    chi, w = O.grid_chi(n, lo, hi)
    assert np.allclose(np.diff(chi), (hi - lo) / (n - 1))
    assert abs(w.sum() - (hi - lo)) < 1e-12 * (hi - lo)
    c = np.array([0.3, -1.1, 0.7, 2.0])
    f = lambda x: c[0] + c[1] * x + c[2] * x ** 2 + c[3] * x ** 3
    F = lambda x: c[0] * x + c[1] * x ** 2 / 2 + c[2] * x ** 3 / 3 + c[3] * x ** 4 / 4
    assert abs(np.dot(w, f(chi)) - (F(hi) - F(lo))) < 1e-13 * abs(F(hi) - F(lo))
    # not exact for quartics (the rule really is Simpson, not something of higher order)
    if n < 20:
        assert abs(np.dot(w, chi ** 4) - (hi ** 5 - lo ** 5) / 5) > 1e-9 * hi ** 5


@pytest.mark.parametrize("n,Rmin", [(32, 0.3), (48, 0.0), (96, 0.3), (7, 0.5)])
def test_fejer1_exact_to_degree_n_minus_1(n, Rmin):
    R, w = O.grid_R(n, Rmin)
    assert np.all(np.diff(R) > 0) and R[0] > Rmin and R[-1] < 1.0
    assert np.all(w > 0)
    assert abs(w.sum() - (1 - Rmin)) < 1e-14
    # the nodes are the first-kind Chebyshev points (Eq. chebpoints) mapped to [Rmin, 1]
    t = np.cos((2 * np.arange(n) + 1) * np.pi / (2 * n))
    assert np.allclose(np.sort(R), np.sort(Rmin + 0.5 * (1 - Rmin) * (t + 1)), atol=1e-15)
    for d in [0, 1, n // 2, n - 1]:
        exact = (1 - Rmin ** (d + 1)) / (d + 1)
        assert abs(np.dot(w, R ** d) - exact) < 1e-13
    # and not beyond: T_d(x(R)) with the first even degree d >= n is integrated with an error
    x = (2 * R - 1 - Rmin) / (1 - Rmin)
    d = n if n % 2 == 0 else n + 1
    exact = 0.5 * (1 - Rmin) * 2.0 / (1.0 - d * d)
    assert abs(np.dot(w, np.cos(d * np.arccos(x))) - exact) > 1e-3 * abs(exact)


def test_k_nodes_are_chebyshev_points_in_log_k():
    n, kmin, kmax = 64, 1e-4, 10.0
    k, x = O.grid_k(n, kmin, kmax)
    assert np.all(np.diff(k) > 0)
    t = np.cos((2 * np.arange(n) + 1) * np.pi / (2 * n))
    assert np.allclose(x, t[::-1], atol=1e-15)
    assert np.allclose(2 * np.log(k / kmin) / np.log(kmax / kmin) - 1, x, atol=1e-13)


def test_prefactors_against_factorials():
    for l in [2, 3, 10, 57]:
        r = math.factorial(l + 2) / math.factorial(l - 2)
        assert abs(O.prefactor("gg", l) - 2 / math.pi) < 1e-16
        assert abs(O.prefactor("gs", l) / (2 / math.pi * math.sqrt(r)) - 1) < 1e-15
        assert abs(O.prefactor("ss", l) / (2 / math.pi * r) - 1) < 1e-15


# ----------------------------------------------------------------------------- Chebyshev interpolant

def _T(m, x):
    return np.cos(m * np.arccos(np.clip(x, -1, 1)))


@pytest.mark.parametrize("N", [8, 16, 64])
def test_interpolant_identity_and_polynomial_exactness(N):
    _, x = O.grid_k(N, 1e-4, 10.0)
    rng = np.random.default_rng(1)
    f = rng.normal(size=N)
    for i in range(N):
        assert O.cheb_interp(f, x[i]) == f[i]
    a = rng.normal(size=N)  # degree N-1 polynomial
    poly = lambda xx: np.polynomial.chebyshev.chebval(xx, a)
    for xx in rng.uniform(-1, 1, 25):
        assert abs(O.cheb_interp(poly(x), xx) - poly(xx)) < 1e-12 * np.abs(a).sum()


def test_aliasing_first_kind():
    """Eq. cheb2 for first-kind points: T_N interpolates to 0, T_{2N-n} to -T_n,
    T_{2N+n} to -T_n and T_{4N-n} to +T_n."""
    N = 16
    _, x = O.grid_k(N, 1e-4, 10.0)
    pts = np.linspace(-0.97, 0.97, 13)
    approx = lambda m, xx: O.cheb_interp(_T(m, x), xx)
    for xx in pts:
        assert abs(approx(N, xx)) < 1e-12
        for n in [1, 3, 13]:
            assert abs(approx(2 * N - n, xx) + _T(n, xx)) < 1e-12
            assert abs(approx(2 * N + n, xx) + _T(n, xx)) < 1e-12
            assert abs(approx(4 * N - n, xx) - _T(n, xx)) < 1e-12


# ----------------------------------------------------------------------------- k-integral

def weber(l, a, b, p):
    """int_0^inf k^2 exp(-p^2 k^2) j_l(ak) j_l(bk) dk = sqrt(pi)/(4p^3) e^{-(a-b)^2/4p^2} e^{-z} i_l(z)."""
    z = a * b / (2 * p * p)
    il_scaled = sp.ive(l + 0.5, z) * np.sqrt(np.pi / (2 * z))
    return np.sqrt(np.pi) / (4 * p ** 3) * np.exp(-(a - b) ** 2 / (4 * p * p)) * il_scaled


@pytest.mark.parametrize("a,b,p", [(50, 40, 10), (100, 90, 5), (300, 280, 12), (2000, 1900, 20),
                                   (1500, 1500, 40), (3000, 2200, 8)])
def test_weber_closed_form_all_types(a, b, p):
    ell = [2, 10, 30, 100, 200]
    ex = np.array([weber(l, a, b, p) for l in ell])
    kmin, kmax = 1e-7, 12.0
    # gg: f = k^2 with P = e^{-p^2k^2}; gs: f = 1 with P = k^2 e^{..}; ss: f = 1/k^2 with P = k^4 e^{..}
    for t, m in (("gg", 0.0), ("gs", 2.0), ("ss", 4.0)):
        w = O.w_points(ell, [t], kmin, kmax, [a], [b], mode=O.P_GAUSS, gauss=(p, m, 1.0), M=64, Phi=10.0)
        got = w[O.types_mask([t]).bit_length() - 1, :, 0]
        scale = np.sqrt(np.pi) / (4 * p ** 3) / max(a * b / (2 * p * p), 1.0)  # size of the integrand
        assert np.all(np.abs(got - ex) <= 1e-10 * np.maximum(np.abs(ex), 1e-3 * scale)), (t, got, ex)


@pytest.mark.parametrize("a,b,p", [(50, 40, 10), (300, 280, 12), (1500, 1500, 40)])
def test_weber_closed_form_real_ell(a, b, p):
    """Weber's closed form holds for any real order: the non-integer path of the k-integral."""
    ell = [2.37, 10.5, 30.9, 100.25, 199.99]
    ex = np.array([weber(l, a, b, p) for l in ell])
    kmin, kmax = 1e-7, 12.0
    for t, m in (("gg", 0.0), ("gs", 2.0), ("ss", 4.0)):
        w = O.w_points(ell, [t], kmin, kmax, [a], [b], mode=O.P_GAUSS, gauss=(p, m, 1.0), M=64, Phi=10.0)
        got = w[O.types_mask([t]).bit_length() - 1, :, 0]
        scale = np.sqrt(np.pi) / (4 * p ** 3) / max(a * b / (2 * p * p), 1.0)
        assert np.all(np.abs(got - ex) <= 1e-10 * np.maximum(np.abs(ex), 1e-3 * scale)), (t, got, ex)


def test_polynomial_P_is_reproduced_exactly():
    """Check (b): for P a polynomial of degree < N in x(k), the interpolant of its
    nodal values is P itself, so nodal mode == exact mode."""
    N = 24
    kmin, kmax = 1e-4, 1.5
    k, x = O.grid_k(N, kmin, kmax)
    rng = np.random.default_rng(7)
    a = rng.normal(size=N) * 0.5 ** np.arange(N)
    nodal = np.polynomial.chebyshev.chebval(x, a)
    ell = [2, 5, 17, 40]
    chi1 = np.array([400.0, 900.0, 1200.0])
    chi2 = np.array([380.0, 610.0, 1190.0])
    w_nod = O.w_points(ell, "gg gs ss".split(), kmin, kmax, chi1, chi2, nc=N, P=nodal, shared=True)
    w_ex = O.w_points(ell, "gg gs ss".split(), kmin, kmax, chi1, chi2, mode=O.P_CHEB, cheb_coef=a,
                      shared=True, M=max(64, 2 * N))
    scale = np.abs(w_ex).max(axis=(1, 2), keepdims=True)
    assert np.all(np.abs(w_nod - w_ex) <= 1e-11 * scale)


def test_w_symmetric_and_converged():
    ell = [2, 20, 60]
    kmin, kmax, N = 1e-4, 2.0, 32
    k, _ = O.grid_k(N, kmin, kmax)
    cosmo = W.Cosmo(2e4)
    nodal = W.p0(k, cosmo)
    w12 = O.w_points(ell, "gg gs ss".split(), kmin, kmax, [1500.0], [1300.0], nc=N, P=nodal, shared=True)
    w21 = O.w_points(ell, "gg gs ss".split(), kmin, kmax, [1300.0], [1500.0], nc=N, P=nodal, shared=True)
    assert np.allclose(w12, w21, rtol=1e-12, atol=0)
    w_fine = O.w_points(ell, "gg gs ss".split(), kmin, kmax, [1500.0], [1300.0], nc=N, P=nodal, shared=True,
                        M=256, Phi=2.5)
    assert np.allclose(w12, w_fine, rtol=1e-11, atol=0)


# ----------------------------------------------------------------------------- outer integrals

def _gauss(x, c, s):
    return np.exp(-0.5 * ((x - c) / s) ** 2) / (math.sqrt(2 * math.pi) * s)


def _graded(n, lo, hi):
    """GL nodes on [lo, hi] graded towards hi: x = hi - (hi-lo) s^3, s in [0,1]."""
    s, ws = np.polynomial.legendre.leggauss(n)
    s = 0.5 * (s + 1)
    ws = 0.5 * ws
    return hi - (hi - lo) * s ** 3, ws * 3 * (hi - lo) * s ** 2


def test_rform_matches_chi1_chi2_square():
    """Check (d): Eq. final_cls (chi-R with symmetrisation) equals Eq. cls-general
    integrated over the full chi1-chi2 square, for kernels that vanish at the
    edges, including the ordering of the bins (C^{AB}_{ij} = C^{BA}_{ji}).
    A smooth spectrum with a Gaussian taper keeps w free of features that the
    two (different) outer quadratures would resolve differently."""
    ell = [2, 12, 30]
    kmin, kmax, N = 1e-4, 0.6, 32
    k, _ = O.grid_k(N, kmin, kmax)
    nodal = 2e4 * k / (1 + (k / 0.02) ** 2.8) * np.exp(-(k / 0.15) ** 2)
    lo, hi = 200.0, 2200.0
    bins = [(1000.0, 110.0), (1250.0, 130.0), (1400.0, 160.0)]  # 2 "g" + 1 "s" bins
    K = lambda xx: np.array([_gauss(xx, c, s) for c, s in bins])
    ng, ns = 2, 1
    types = "gg gs ss".split()
    # chi-R form on fine rules
    xg, wg = np.polynomial.legendre.leggauss(80)
    chi = lo + (hi - lo) * 0.5 * (xg + 1)
    wchi = 0.5 * (hi - lo) * wg
    R, wR = _graded(96, 0.05, 1.0)
    c1 = np.repeat(chi, len(R))
    c2 = (chi[:, None] * R[None, :]).ravel()
    w = O.w_points(ell, types, kmin, kmax, c1, c2, nc=N, P=nodal, shared=True)
    C_r = O.sum_rform(chi, wchi, wR, ng, ns, K(chi), K(c2).reshape(3, len(chi), len(R)), ell, types, w)
    # full square: for each chi1, chi2 on [lo, chi1] and [chi1, hi], graded towards the diagonal
    P1, P2, WW = [], [], []
    for x1, w1 in zip(chi, wchi):
        a, wa = _graded(60, lo, x1)
        b, wb = _graded(60, hi, x1)
        P1 += [x1] * 120
        P2 += list(a) + list(b)
        WW += list(w1 * wa) + list(-w1 * wb)
    P1, P2, WW = map(np.array, (P1, P2, WW))
    w2 = O.w_points(ell, types, kmin, kmax, P1, P2, nc=N, P=nodal, shared=True)
    C_sq = O.sum_points(WW, ng, ns, K(P1), K(P2), ell, types, w2)
    assert np.all(np.abs(C_r - C_sq) <= 1e-4 * np.abs(C_sq) + 1e-9 * np.abs(C_sq).max()), \
        np.abs(C_r / C_sq - 1).max()
    # ordering of bins: swap the two clustering bins -> the gg cross spectrum is unchanged
    Ksw = lambda xx: K(xx)[[1, 0, 2]]
    C_sw = O.sum_rform(chi, wchi, wR, ng, ns, Ksw(chi), Ksw(c2).reshape(3, len(chi), len(R)), ell, types, w)
    assert np.array_equal(C_sw[1], C_r[1])          # gg (0,1) == gg (1,0)
    assert np.array_equal(C_sw[0], C_r[2])          # autos swap places
    assert np.array_equal(C_sw[3], C_r[4])          # gs (0,s) <-> (1,s)


def test_limber_limit_at_high_ell():
    """Check (c): the relative gap between the exact (continuous chi-R) C_ell and
    the first-order Limber C_ell (Sec. "The Limber approximation", with the
    closure relation int dk k^2 j_l(k chi1) j_l(k chi2) = pi/(2 chi1^2) delta(chi1-chi2))
    shrinks like nu^-2, nu = l + 1/2, for all three spectra.  A pure power law
    P = k^-2 keeps the coefficient of nu^-2 independent of ell.  This pins the
    absolute normalisation of the chi-R form (Jacobian, symmetrisation, N_t,
    f_t): any slip there leaves an O(1) gap that does not shrink."""
    ell = [25, 50, 100]
    kmin, kmax, N = 1e-4, 1.0, 64
    k, _ = O.grid_k(N, kmin, kmax)
    nodal = k ** -2.0
    lo, hi = 900.0, 2300.0
    types = "gg gs ss".split()
    K = lambda xx: np.array([_gauss(xx, 1600.0, 150.0)] * 2)   # one "g" and one "s" bin
    xg, wg = np.polynomial.legendre.leggauss(56)
    chi = lo + (hi - lo) * 0.5 * (xg + 1)
    wchi = 0.5 * (hi - lo) * wg
    R, wR = _graded(96, 0.4, 1.0)
    c1 = np.repeat(chi, len(R))
    c2 = (chi[:, None] * R[None, :]).ravel()
    w = O.w_points(ell, types, kmin, kmax, c1, c2, nc=N, P=nodal, shared=True)
    C_ex = O.sum_rform(chi, wchi, wR, 1, 1, K(chi), K(c2).reshape(2, len(chi), len(R)), ell, types, w)
    C_lb = O.limber(chi, wchi, 1, 1, K(chi), ell, types, kmin, kmax, nodal)
    gap = np.abs(C_ex / C_lb - 1)
    nu2 = (np.array(ell) + 0.5) ** 2
    for p in range(3):
        assert gap[p, 0] < 0.2
        r1, r2 = gap[p, 0] / gap[p, 1], gap[p, 1] / gap[p, 2]
        assert 2.5 < r1 < 5.0 and 3.0 < r2 < 5.0, (types[p], gap[p])
        # and nu^2 * gap is nearly constant between the two highest multipoles
        assert 0.7 < (gap[p, 2] * nu2[2]) / (gap[p, 1] * nu2[1]) < 1.3
