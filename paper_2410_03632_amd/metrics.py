"""Accuracy metric of the paper's benchmark comparison (Sec. "Challenge set-up", Eq. dchi).

    Delta chi^2 = sum_b N_b Tr[(S(l_b)^-1 Delta C(l_b))^2],   N_b = f_sky/2 sum_{l in b} (2 l + 1),

with S = C + N the symmetric (n_g + n_s) x (n_g + n_s) matrix of the benchmark's auto and
cross spectra (clustering bins first) plus shot / shape noise (diagonal), and Delta C the same
matrix of differences.  The paper prints S with an extra factor sqrt(2 / ((2l+1) Delta l f_sky));
together with N_b that counts the modes twice, and the equivalence the paper cites with the
quadratic form Delta x^T Cov^-1 Delta x of the Gaussian covariance
Cov[C_ij, C_kl] = (S_ik S_jl + S_il S_jk) / (2 N_b) holds for the form above (pinned in the
tests), which is the one implemented.

Each multipole of the plan is its own band, Delta l_b = half the distance between its
neighbours (the end bands extend by their one neighbour distance).
"""
from __future__ import annotations

import math

import numpy as np

from .workloads import pair_list

ARCMIN2_PER_SR = (180.0 * 60.0 / math.pi) ** 2


def g16_err(C, Cref, n_g, n_s, types=("gg", "gs", "ss")):
    """Per-element relative error |C - Cref| / max(|Cref|, 1e-3 sqrt(|Cref_ii Cref_jj|)) of
    spectra [pair][ell]: cross spectra of separated bins pass through zero, so their error is
    measured against the geometric mean of the two auto spectra below a thousandth of it."""
    C = np.asarray(C, dtype=np.float64)
    Cref = np.asarray(Cref, dtype=np.float64)
    pairs = pair_list(n_g, n_s, types)
    auto = {i: p for p, (t, i, j) in enumerate(pairs) if i == j}
    out = np.empty_like(C)
    for p, (t, i, j) in enumerate(pairs):
        den = np.abs(Cref[p])
        if i in auto and j in auto:
            den = np.maximum(den, 1e-3 * np.sqrt(np.abs(Cref[auto[i]] * Cref[auto[j]])))
        den = np.where(den > 0, den, 1.0)
        out[p] = np.abs(C[p] - Cref[p]) / den
    return out


def error_by_pair(C, Cref, n_g, n_s, ell, worst=3):
    """Error summary of one set of spectra against a reference (the g16_err metric): the largest
    error of each pair type, and the `worst` pairs with the multipole where each peaks."""
    e = g16_err(C, Cref, n_g, n_s)
    pairs = pair_list(n_g, n_s)
    by_type = {}
    for p, (t, i, j) in enumerate(pairs):
        by_type[t] = max(by_type.get(t, 0.0), float(e[p].max()))
    peak = e.max(axis=1)
    order = np.argsort(-peak)[:worst]
    rows = [{"pair": "%s %d-%d" % (pairs[p][0], pairs[p][1], pairs[p][2]), "max": float(peak[p]),
             "ell": float(np.asarray(ell)[int(np.argmax(e[p]))])} for p in order]
    return {"max": float(e.max()), "by_type": by_type, "worst_pairs": rows}


def spectra_matrix(C_pairs, n_g, n_s, pairs):
    """[n_ell, nb, nb] symmetric matrices from C[pair][ell] with pairs = list of (type, i, j)."""
    nb = n_g + n_s
    C_pairs = np.asarray(C_pairs, dtype=np.float64)
    M = np.zeros((C_pairs.shape[1], nb, nb))
    for p, (_, i, j) in enumerate(pairs):
        M[:, i, j] = C_pairs[p]
        M[:, j, i] = C_pairs[p]
    return M


def noise(n_g, n_s, sigma_e=0.28, n_src=27.0, n_lens=40.0):
    """Diagonal noise [nb]: 1/n per clustering bin and sigma_e^2/n per shear bin, with the
    total densities (per arcmin^2) split evenly over the bins, in sr units."""
    N = np.zeros(n_g + n_s)
    if n_g:
        N[:n_g] = 1.0 / (n_lens / n_g * ARCMIN2_PER_SR)
    if n_s:
        N[n_g:] = sigma_e ** 2 / (n_src / n_s * ARCMIN2_PER_SR)
    return N


def band_widths(ell):
    ell = np.asarray(ell, dtype=np.float64)
    if ell.size == 1:
        return np.ones(1)
    d = np.diff(ell)
    w = np.empty_like(ell)
    w[1:-1] = 0.5 * (d[:-1] + d[1:])
    w[0], w[-1] = d[0], d[-1]
    return w


def delta_chi2(C, C_bench, ell, n_g, n_s, pairs, f_sky=0.4, N=None, ell_max=None):
    """Delta chi^2 of spectra C against the benchmark C_bench (both [pair][ell]); with ell_max,
    only the bands with l < ell_max count (the paper's requirement is stated for l < 200).  Band
    widths always come from the full multipole list."""
    ell = np.asarray(ell, dtype=np.float64)
    S = spectra_matrix(C_bench, n_g, n_s, pairs)
    if N is None:
        N = noise(n_g, n_s)
    S = S + np.diag(N)[None]
    dC = spectra_matrix(np.asarray(C) - np.asarray(C_bench), n_g, n_s, pairs)
    Nb = 0.5 * f_sky * (2 * ell + 1) * band_widths(ell)
    tot = 0.0
    for b in range(ell.size):
        if ell_max is not None and ell[b] >= ell_max:
            continue
        X = np.linalg.solve(S[b], dC[b])
        tot += Nb[b] * np.trace(X @ X)
    return float(tot)
