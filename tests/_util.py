"""Shared test helpers: the parity metric and small builders (test infrastructure)."""
import numpy as np

from paper_2410_03632_amd import workloads as W


def g16_err(C, Cref, n_g, n_s, types=("gg", "gs", "ss"), ell_axis_len=None):
    """Per-element |C - Cref| / max(|Cref|, 1e-3 sqrt(|Cref_ii Cref_jj|)); the floor
    handles cross spectra that pass through zero.  C, Cref: [pairs, ell]."""
    C = np.asarray(C, dtype=np.float64)
    Cref = np.asarray(Cref, dtype=np.float64)
    pairs = W.pair_list(n_g, n_s, types)
    auto = {}
    for p, (t, i, j) in enumerate(pairs):
        if i == j:
            auto[i] = p
    out = np.empty_like(C)
    for p, (t, i, j) in enumerate(pairs):
        den = np.abs(Cref[p])
        if i in auto and j in auto:
            den = np.maximum(den, 1e-3 * np.sqrt(np.abs(Cref[auto[i]] * Cref[auto[j]])))
        den = np.where(den > 0, den, 1.0)
        out[p] = np.abs(C[p] - Cref[p]) / den
    return out
