"""ctypes wrapper of the FP64 CPU oracle (``oracle/blast_oracle.c``).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The HIP library and
its Python binding never import it, and it imports nothing from them.

Every function mirrors a C entry point of the oracle; the docstrings there cite the
passages of arXiv:2410.03632 each one follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "blast_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

GG, GS, SS = 1, 2, 4
P_NODAL, P_GAUSS, P_CHEB = 0, 1, 2
TYPE_OF = {"gg": GG, "gs": GS, "ss": SS}

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.or_gl16.argtypes = [dp, dp]
        L.or_grid_chi.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp]
        L.or_grid_R.argtypes = [C.c_int, C.c_double, dp, dp]
        L.or_grid_k.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp]
        L.or_prefactor.argtypes = [C.c_int, C.c_double]
        L.or_prefactor.restype = C.c_double
        L.or_sph_jn.argtypes = [C.c_int, C.c_double, dp]
        L.or_sph_jnu.argtypes = [C.c_double, C.c_double]
        L.or_sph_jnu.restype = C.c_double
        L.or_cheb_interp.argtypes = [C.c_int, dp, C.c_double]
        L.or_cheb_interp.restype = C.c_double
        L.or_w_points.argtypes = [C.c_int, dp, C.c_int, C.c_double, C.c_double, C.c_int, C.c_long,
                                  dp, dp, C.c_int, dp, C.c_long, C.c_int, C.c_double, C.c_double,
                                  C.c_double, C.c_int, C.c_double, dp, C.c_int]
        L.or_sum_rform.argtypes = [C.c_int, C.c_int, dp, dp, dp, C.c_int, C.c_int, dp, dp, C.c_int, dp,
                                   C.c_int, dp, dp]
        L.or_sum_points.argtypes = [C.c_long, dp, C.c_int, C.c_int, dp, dp, C.c_int, dp, C.c_int, dp, dp]
        L.or_limber.argtypes = [C.c_int, dp, dp, C.c_int, C.c_int, dp, C.c_int, dp, C.c_int, C.c_double,
                                C.c_double, C.c_int, dp, dp]
        L.or_cl_grid.argtypes = [C.c_int, dp, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int,
                                 dp, dp, dp, dp, dp, C.c_int, C.c_int, dp, dp, C.c_int, C.c_double,
                                 C.c_double, C.c_int, dp, dp, dp, ip, C.c_int]
        L.or_npairs.argtypes = [C.c_int, C.c_int, C.c_int]
        L.or_pair.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, ip, ip, ip]
        L.or_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _ell(a):
    """Multipoles as FP64 (integer or not); the oracle takes one recurrence for all of them
    when they are all integers, and a real-order evaluation per multipole otherwise."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def types_mask(types) -> int:
    if isinstance(types, int):
        return types
    m = 0
    for t in types:
        m |= TYPE_OF[t]
    return m


# --------------------------------------------------------------------------- grids

def gl16():
    x = np.empty(16)
    w = np.empty(16)
    lib().or_gl16(_d(x)[1], _d(w)[1])
    return x, w


def grid_chi(n, lo, hi):
    chi, w = np.empty(n), np.empty(n)
    if lib().or_grid_chi(n, lo, hi, chi.ctypes.data_as(C.POINTER(C.c_double)),
                         w.ctypes.data_as(C.POINTER(C.c_double))):
        raise ValueError("bad chi grid")
    return chi, w


def grid_R(n, Rmin):
    R, w = np.empty(n), np.empty(n)
    if lib().or_grid_R(n, Rmin, R.ctypes.data_as(C.POINTER(C.c_double)),
                       w.ctypes.data_as(C.POINTER(C.c_double))):
        raise ValueError("bad R grid")
    return R, w


def grid_k(n, kmin, kmax):
    k, x = np.empty(n), np.empty(n)
    if lib().or_grid_k(n, kmin, kmax, k.ctypes.data_as(C.POINTER(C.c_double)),
                       x.ctypes.data_as(C.POINTER(C.c_double))):
        raise ValueError("bad k grid")
    return k, x


def prefactor(t, ell):
    return lib().or_prefactor(types_mask([t]) if isinstance(t, str) else t, float(ell))


def sph_jn(lmax, x):
    out = np.empty(lmax + 1)
    lib().or_sph_jn(int(lmax), float(x), out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def sph_jnu(nu, x):
    """j_nu(x) for real order nu >= 0 (Miller's recurrence normalised by Neumann's series)."""
    return lib().or_sph_jnu(float(nu), float(x))


def cheb_interp(f_nodes, x):
    f, fp = _d(f_nodes)
    return lib().or_cheb_interp(len(f), fp, float(x))


def npairs(ng, ns, types="gg gs ss".split()):
    return lib().or_npairs(ng, ns, types_mask(types))


def pair(p, ng, ns, types="gg gs ss".split()):
    t, i, j = C.c_int(), C.c_int(), C.c_int()
    lib().or_pair(p, ng, ns, types_mask(types), C.byref(t), C.byref(i), C.byref(j))
    return {GG: "gg", GS: "gs", SS: "ss"}[t.value], i.value, j.value


# --------------------------------------------------------------------------- k-integrals

def w_points(ell, types, kmin, kmax, chi1, chi2, *, nc=0, P=None, shared=False, mode=P_NODAL,
             cheb_coef=None, gauss=(0.0, 0.0, 1.0), M=None, Phi=10.0, nthreads=0):
    """w[t][il][m] = int_{kmin}^{kmax} dk f_t(k) P(k; chi1_m, chi2_m) j_l(k chi1_m) j_l(k chi2_m).

    mode P_NODAL: P = interpolant of nodal values (P[m, :nc], or one shared row);
    mode P_CHEB : P = sum a_n T_n(x(k)) with coefficients cheb_coef[m, :d] (or shared);
    mode P_GAUSS: P = amp k^m exp(-(p k)^2), gauss = (p, m, amp)."""
    ell, ellp = _ell(ell)
    chi1, c1p = _d(np.atleast_1d(chi1))
    chi2, c2p = _d(np.atleast_1d(chi2))
    npts = len(chi1)
    nl = len(ell)
    w = np.zeros((3, nl, npts))
    pd = 0
    if mode == P_NODAL:
        data, datap = _d(P)
        stride = 0 if shared else nc
    elif mode == P_CHEB:
        data, datap = _d(cheb_coef)
        pd = data.shape[-1]
        stride = 0 if shared else pd
    else:
        data, datap = None, None
        stride = 0
    if M is None:
        M = max(64, 2 * max(nc, pd, 1))
    rc = lib().or_w_points(nl, ellp, types_mask(types), kmin, kmax, int(nc), npts, c1p, c2p, mode,
                           datap, stride, pd, gauss[0], gauss[1], gauss[2], int(M), float(Phi),
                           w.ctypes.data_as(C.POINTER(C.c_double)), nthreads)
    if rc:
        raise RuntimeError("or_w_points failed (%d)" % rc)
    return w


# --------------------------------------------------------------------------- outer sums

def sum_rform(chi, wchi, wR, n_g, n_s, Kchi, Kchi2, ell, types, w):
    chi, cp = _d(chi)
    wchi, wcp = _d(wchi)
    wR, wrp = _d(wR)
    Kchi, kp = _d(Kchi)
    Kchi2, k2p = _d(Kchi2)
    ell, ellp = _ell(ell)
    w, wp = _d(w)
    tm = types_mask(types)
    C_out = np.zeros((npairs(n_g, n_s, tm), len(ell)))
    lib().or_sum_rform(len(chi), len(wR), cp, wcp, wrp, n_g, n_s, kp, k2p, len(ell), ellp, tm, wp,
                       C_out.ctypes.data_as(C.POINTER(C.c_double)))
    return C_out


def sum_points(W, n_g, n_s, K1, K2, ell, types, w):
    W, Wp = _d(W)
    K1, k1p = _d(K1)
    K2, k2p = _d(K2)
    ell, ellp = _ell(ell)
    w, wp = _d(w)
    tm = types_mask(types)
    C_out = np.zeros((npairs(n_g, n_s, tm), len(ell)))
    lib().or_sum_points(len(W), Wp, n_g, n_s, k1p, k2p, len(ell), ellp, tm, wp,
                        C_out.ctypes.data_as(C.POINTER(C.c_double)))
    return C_out


def limber(chi, wchi, n_g, n_s, K, ell, types, kmin, kmax, p_nodal):
    chi, cp = _d(chi)
    wchi, wcp = _d(wchi)
    K, kp = _d(K)
    ell, ellp = _ell(ell)
    pn, pnp = _d(p_nodal)
    tm = types_mask(types)
    C_out = np.zeros((npairs(n_g, n_s, tm), len(ell)))
    rc = lib().or_limber(len(chi), cp, wcp, n_g, n_s, kp, len(ell), ellp, tm, kmin, kmax, len(pn), pnp,
                         C_out.ctypes.data_as(C.POINTER(C.c_double)))
    if rc:
        raise RuntimeError("or_limber failed")
    return C_out


def cl_grid(ell, types, kmin, kmax, nc, chi, wchi, R, wR, P, n_g, n_s, Kchi, Kchi2, *,
            M0=None, Phi0=10.0, tol=1e-10, maxlev=4, want_w=False, nthreads=0):
    """The discrete target C[p][il] on the (chi, R) grid with its self-convergence
    estimate.  Returns (C, err, levels, w or None)."""
    ell, ellp = _ell(ell)
    chi, cp = _d(chi)
    wchi, wcp = _d(wchi)
    R, rp = _d(R)
    wR, wrp = _d(wR)
    P, pp = _d(P)
    Kchi, kp = _d(Kchi)
    Kchi2, k2p = _d(Kchi2)
    tm = types_mask(types)
    na, nb = len(chi), len(R)
    if P.size != na * nb * nc:
        raise ValueError("P must hold n_chi*n_R*n_cheb values")
    if M0 is None:
        M0 = max(64, 2 * nc)
    nl = len(ell)
    C_out = np.zeros((npairs(n_g, n_s, tm), nl))
    w = np.zeros((3, nl, na * nb)) if want_w else None
    err = C.c_double()
    lev = C.c_int()
    rc = lib().or_cl_grid(nl, ellp, tm, kmin, kmax, nc, na, nb, cp, wcp, rp, wrp, pp, n_g, n_s, kp, k2p,
                          int(M0), float(Phi0), float(tol), int(maxlev),
                          C_out.ctypes.data_as(C.POINTER(C.c_double)),
                          w.ctypes.data_as(C.POINTER(C.c_double)) if want_w else None,
                          C.byref(err), C.byref(lev), nthreads)
    if rc:
        raise RuntimeError("or_cl_grid failed (%d)" % rc)
    return C_out, err.value, lev.value, w


def max_threads():
    return lib().or_max_threads()
