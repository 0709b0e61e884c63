"""GPU parity for non-integer multipoles.

The challenge the paper evaluates on samples C_ell at log-spaced multipoles that are not
integers; the method itself only needs j_l of real order in the basis precompute (Eq. t_tilde)
and N_t(l), k = (l + 1/2)/chi in the Limber pieces.  The plan takes such lists; the oracle's
real-order Bessel function is pinned against mpmath and Weber's closed form on the CPU.
"""
import os

import numpy as np
import pytest

import oracle as O
from oracle import limber_approx as LA
from paper_2410_03632_amd import blast as B
from paper_2410_03632_amd import workloads as W
from _util import g16_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ALL = ("gg", "gs", "ss")

# (grid, multipoles): log-spaced reals with integer end points (a fractional part of 0 in a
# non-integer list), a ragged grid, and one long run of equal fractional part
CASES = [
    (dict(n_ell=6, ell_max=40, chi_min=200.0, chi_max=800.0, k_max=0.3), W.real_ell_list(6, 2.0, 40.0)),
    (dict(n_ell=17, ell_max=90, n_chi=9, n_R=7, n_cheb=40, k_max=0.5, chi_min=200.0, chi_max=900.0),
     W.real_ell_list(17, 2.3, 90.7)),
    (dict(n_ell=8, ell_max=40, n_chi=8, n_R=6, n_cheb=32, k_max=0.3, chi_min=200.0, chi_max=800.0),
     2.5 + 5.0 * np.arange(8)),
]


def _dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).cuda()


def _run(plan, inp, precision="fp64", p32=False):
    P = _dev(inp.P[None], torch.float32 if p32 else torch.float64)
    C = plan.forward(P, _dev(inp.Kchi[None]), _dev(inp.Kchi2[None]), inp.n_g, inp.n_s, precision=precision)
    torch.cuda.synchronize()
    return C.cpu().numpy()[0]


@pytest.fixture(scope="module", params=range(len(CASES)))
def case(request):
    kw, ell = CASES[request.param]
    cfg = W.tiny_config(**kw)
    print("real-ell case", request.param, np.round(ell, 4).tolist(), flush=True)
    plan = B.plan_for_config(cfg, precisions=("fp64", "fp32"), ell=ell)
    inp = W.make_inputs(cfg, W.seed_for(11, request.param), plan.k_nodes, plan.chi, plan.R)
    chi, wchi = O.grid_chi(cfg.n_chi, cfg.chi_min, cfg.chi_max)
    R, wR = O.grid_R(cfg.n_R, cfg.R_min)
    Cor, err, _, _ = O.cl_grid(ell, ALL, cfg.k_min, cfg.k_max, cfg.n_cheb, chi, wchi, R, wR, inp.P, cfg.n_g,
                               cfg.n_s, inp.Kchi, inp.Kchi2)
    assert err < 1e-9
    yield cfg, ell, plan, inp, Cor
    plan.close()


def test_plan_keeps_real_multipoles(case):
    cfg, ell, plan, inp, Cor = case
    assert plan.ell.dtype == np.float64 and np.array_equal(plan.ell, ell)


def test_real_ell_fp64_matches_oracle(case):
    cfg, ell, plan, inp, Cor = case
    e = g16_err(_run(plan, inp, "fp64"), Cor, cfg.n_g, cfg.n_s)
    print("fp64 max err", e.max(), flush=True)
    assert e.max() <= 1e-6


def test_real_ell_fp32_matches_oracle(case):
    cfg, ell, plan, inp, Cor = case
    e = g16_err(_run(plan, inp, "fp32", p32=True), Cor, cfg.n_g, cfg.n_s)
    print("fp32 max err", e.max(), flush=True)
    assert e.max() <= 1e-3


def test_integer_members_of_a_real_list_match_the_integer_plan():
    """Integer multipoles inside a non-integer list go through the real-order routine (a run of
    fractional part 0 with Hankel seeds or Neumann normalisation); an all-integer plan takes the
    integer recurrence (closed-form j_0, j_1).  Their basis rows must agree."""
    cfg = W.tiny_config(n_ell=3, ell_max=40, chi_min=200.0, chi_max=800.0, k_max=0.3)
    mixed = np.array([2.0, 3.5, 9.0, 17.25, 40.0])
    pi = B.plan_for_config(cfg, precisions=("fp64",), ell=[2, 9, 40])
    pm = B.plan_for_config(cfg, precisions=("fp64",), ell=mixed)
    try:
        N = cfg.n_cheb
        worst = 0.0
        for a, b in [(0, 0), (cfg.n_chi // 2, cfg.n_R - 1), (cfg.n_chi - 1, cfg.n_R // 2)]:
            ti = pi.basis_point(a, b).reshape(3, 3, -1)[:, :, :N]
            tm = pm.basis_point(a, b).reshape(3, 5, -1)[:, [0, 2, 4], :N]
            scale = np.abs(ti).max(axis=2, keepdims=True)
            worst = max(worst, float((np.abs(tm - ti) / scale).max()))
        print("integer vs real-order rows: max rel diff", worst, flush=True)
        assert worst <= 1e-11
    finally:
        pi.close()
        pm.close()


def test_real_ell_limber_matches_oracle(case):
    """Limber and extended Limber at non-integer multipoles (k = (l + 1/2)/chi, N_t(l) real)."""
    cfg, ell, plan, inp, Cor = case
    if len(plan.chi) < 5:
        pytest.skip("extended Limber needs five chi nodes")
    chi = plan.chi
    kl = plan.limber_k()
    Pl = W.p_limber(kl, chi, inp.cosmo)
    for order in (1, 2):
        C = plan.limber(_dev(Pl[None]), _dev(inp.Kchi[None]), cfg.n_g, cfg.n_s, order=order)
        torch.cuda.synchronize()
        ref = LA.cl_limber(ell, chi, plan.w_chi, inp.Kchi, cfg.n_g, cfg.n_s, Pl, order=order)
        got = C.cpu().numpy()[0]
        scale = np.abs(ref).max(axis=-1, keepdims=True)
        assert np.all(np.abs(got - ref) <= 1e-11 * np.abs(ref) + 1e-13 * scale), (order, np.abs(got / ref - 1).max())


def test_real_ell_plan_save_load(case, tmp_path):
    cfg, ell, plan, inp, Cor = case
    path = os.path.join(str(tmp_path), "real.blastplan")
    plan.save(path)
    p2 = B.Plan.load(path, precisions=("fp64",))
    try:
        assert np.array_equal(p2.ell, plan.ell)
        assert np.array_equal(_run(p2, inp, "fp64"), _run(plan, inp, "fp64"))
    finally:
        p2.close()
