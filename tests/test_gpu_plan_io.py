"""GPU checks of the basis checkpoint (blast_plan_save / blast_plan_load).

The basis of Eq. t_tilde is cosmology-independent and computed once; a plan rebuilt from
its file must reproduce the original plan bitwise (same FP64 basis, same derived
reduced-precision copies, same grids), and a damaged file must be refused."""
import os

import numpy as np
import pytest

from paper_2410_03632_amd import blast as B
from paper_2410_03632_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def saved(tmp_path_factory):
    cfg = W.tiny_config(n_ell=17, ell_max=90, n_chi=9, n_R=7, n_cheb=40, k_max=1.2)
    plan = B.plan_for_config(cfg, precisions=("fp64", "fp32", "bf16x3"))
    path = str(tmp_path_factory.mktemp("plan") / "tiny.blastplan")
    plan.save(path)
    inp = W.make_inputs(cfg, W.seed_for(9, 77), plan.k_nodes, plan.chi, plan.R)
    yield cfg, plan, path, inp
    plan.close()


def _fwd(plan, cfg, inp, prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    P = torch.as_tensor(inp.P[None], dtype=dt).cuda()
    K1 = torch.as_tensor(inp.Kchi[None]).cuda()
    K2 = torch.as_tensor(inp.Kchi2[None]).cuda()
    return plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, precision=prec).cpu().numpy()


def test_loaded_plan_is_bitwise_the_saved_plan(saved):
    cfg, plan, path, inp = saved
    q = B.Plan.load(path)
    try:
        for name in ("ell", "chi", "w_chi", "R", "w_R", "k_nodes"):
            assert np.array_equal(getattr(q, name), getattr(plan, name)), name
        assert (q.k_min, q.k_max, q.n_cheb, q.types, q.rows, q.nc_pad) == \
               (plan.k_min, plan.k_max, plan.n_cheb, plan.types, plan.rows, plan.nc_pad)
        assert q.basis_bytes == plan.basis_bytes
        for a, b in [(0, 0), (4, 3), (8, 6)]:
            assert np.array_equal(q.basis_point(a, b), plan.basis_point(a, b))
        for prec in ("fp64", "fp32", "bf16x3"):
            assert np.array_equal(_fwd(q, cfg, inp, prec), _fwd(plan, cfg, inp, prec)), prec
    finally:
        q.close()


def test_load_with_fewer_precisions(saved):
    cfg, plan, path, inp = saved
    q = B.Plan.load(path, precisions=("fp64",))
    try:
        assert q.basis_bytes[1] == 0 and q.basis_bytes[3] == 0
        assert np.array_equal(_fwd(q, cfg, inp, "fp64"), _fwd(plan, cfg, inp, "fp64"))
        with pytest.raises(B.BlastError) as e:
            _fwd(q, cfg, inp, "fp32")
        assert e.value.status == B.E_INVALID       # precision not resident
    finally:
        q.close()


@pytest.mark.parametrize("damage", ["flip_basis", "flip_grid", "truncate", "checksum"])
def test_damaged_file_is_refused(saved, tmp_path, damage):
    cfg, plan, path, inp = saved
    raw = bytearray(open(path, "rb").read())
    if damage == "flip_basis":
        raw[len(raw) // 2] ^= 0x10
    elif damage == "flip_grid":
        raw[8 + 32 + 24 + 4 * plan.n_ell + 3] ^= 0x01    # a chi node
    elif damage == "truncate":
        raw = raw[:len(raw) - 1000]
    else:
        raw[-1] ^= 0xFF
    bad = str(tmp_path / "bad.blastplan")
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(B.BlastError) as e:
        B.Plan.load(bad)
    assert e.value.status == B.E_INVALID
