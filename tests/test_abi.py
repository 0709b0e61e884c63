"""CPU checks of the C ABI: the library loads, exports every declared entry point,
its host-side grids agree with the oracle's independently written ones, and bad
plan descriptors are rejected before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2410_03632_amd import blast as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "blast_hip.h")).read()
    return sorted(set(re.findall(r"\b(blast_[A-Za-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    decl = declared_symbols()
    assert len(decl) >= 12
    for name in decl:
        assert hasattr(L, name), name
    assert set(decl) == set(B.EXPORTS)
    assert "gfx950" in B.version()


@pytest.mark.parametrize("n", [4, 5, 64, 96, 256])
def test_chi_grid_matches_oracle(n):
    a = B.grid_chi_simpson(n, 20.0, 4500.0)
    b = O.grid_chi(n, 20.0, 4500.0)
    assert np.allclose(a[0], b[0], rtol=1e-15, atol=0)
    assert np.allclose(a[1], b[1], rtol=1e-13, atol=0)


@pytest.mark.parametrize("n,Rmin", [(7, 0.5), (32, 0.3), (96, 0.3), (48, 0.0)])
def test_R_grid_matches_oracle(n, Rmin):
    a = B.grid_R_fejer(n, Rmin)
    b = O.grid_R(n, Rmin)
    assert np.allclose(a[0], b[0], rtol=1e-15, atol=1e-16)
    assert np.allclose(a[1], b[1], rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("n", [2, 24, 64, 128])
def test_k_nodes_match_oracle(n):
    a = B.grid_k_cheb(n, 1e-4, 10.0)
    b, _ = O.grid_k(n, 1e-4, 10.0)
    assert np.allclose(a, b, rtol=1e-14, atol=0)


def test_grid_helpers_reject_bad_input():
    with pytest.raises(B.BlastError) as e:
        B.grid_chi_simpson(3, 0.0, 1.0)
    assert e.value.status == B.E_INVALID
    with pytest.raises(B.BlastError):
        B.grid_R_fejer(8, 1.0)
    with pytest.raises(B.BlastError):
        B.grid_k_cheb(8, 0.0, 1.0)


def _desc(**kw):
    ell = np.array(kw.get("ell", [2, 5, 9]), dtype=np.float64)
    chi = np.array(kw.get("chi", [100.0, 200.0, 300.0, 400.0]))
    w = np.ones_like(chi)
    R = np.array(kw.get("R", [0.5, 0.9]))
    wR = np.ones_like(R)
    keep = (ell, chi, w, R, wR)
    d = B.PlanDesc(len(ell), ell.ctypes.data_as(C.POINTER(C.c_double)), len(chi),
                   chi.ctypes.data_as(C.POINTER(C.c_double)), w.ctypes.data_as(C.POINTER(C.c_double)),
                   len(R), R.ctypes.data_as(C.POINTER(C.c_double)), wR.ctypes.data_as(C.POINTER(C.c_double)),
                   kw.get("kmin", 1e-4), kw.get("kmax", 1.0), kw.get("n_cheb", 16), kw.get("types", 7),
                   kw.get("prec", 1), 0, 0.0)
    return d, keep


@pytest.mark.parametrize("bad", [dict(ell=[2, 2, 5]), dict(ell=[1, 4]), dict(ell=[2.5, 2.5]), dict(ell=[1.99, 3.0]),
                                 dict(ell=[2.0, float("nan")]), dict(ell=[2.0, 4096.5]), dict(chi=[0.0, 1.0, 2.0, 3.0]),
                                 dict(R=[0.5, 1.2]), dict(kmin=2.0, kmax=1.0), dict(n_cheb=1),
                                 dict(n_cheb=300), dict(types=0), dict(types=8), dict(prec=32)])
def test_plan_create_rejects_bad_descriptor(bad):
    d, keep = _desc(**bad)
    h = C.c_void_p()
    st = B.lib().blast_plan_create(C.byref(d), 0, C.byref(h))
    assert st == B.E_INVALID
    assert not h.value
    assert len(B.lib().blast_last_error()) > 0


@pytest.mark.parametrize("content", [b"", b"not a plan file at all", b"BLASTPL1" + b"\x07\x00\x00\x00" * 8])
def test_plan_load_rejects_foreign_files(tmp_path, content):
    """A file that is not a plan checkpoint is refused before any device work."""
    path = tmp_path / "x.blastplan"
    path.write_bytes(content)
    with pytest.raises(B.BlastError) as e:
        B.Plan.load(str(path))
    assert e.value.status == B.E_INVALID


def test_plan_load_missing_file(tmp_path):
    with pytest.raises(B.BlastError) as e:
        B.Plan.load(str(tmp_path / "absent.blastplan"))
    assert e.value.status == B.E_INVALID
