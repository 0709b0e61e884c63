"""GPU parity: the HIP path against the FP64 CPU oracle on the same seeded inputs.

Every test calls the library through its C ABI (``paper_2410_03632_amd.blast``) and
the oracle through ``oracle`` on identical P grids and kernels.  The bar is the
relative error of ``metrics.g16_err`` (|dC| / max(|C|, 1e-3 sqrt(C_ii C_jj))):
<= 1e-6 for the FP64 path, <= 1e-3 for FP32 and FP16X3, and the bounds blast_hip.h states
for BF16X3 and plain BF16.
"""
import json
import os
import time

import numpy as np
import pytest

import oracle as O
from paper_2410_03632_amd import blast as B
from paper_2410_03632_amd import workloads as W
from _util import g16_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ALL = ("gg", "gs", "ss")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).cuda()


def _run(plan, inp, precision="fp64", p32=False, **kw):
    P = _dev(inp.P[None], torch.float32 if p32 else torch.float64)
    C = plan.forward(P, _dev(inp.Kchi[None]), _dev(inp.Kchi2[None]), inp.n_g, inp.n_s, precision=precision, **kw)
    torch.cuda.synchronize()
    return C.cpu().numpy()[0]


def _oracle(cfg, inp, ell=None, types=ALL):
    chi, wchi = O.grid_chi(cfg.n_chi, cfg.chi_min, cfg.chi_max)
    R, wR = O.grid_R(cfg.n_R, cfg.R_min)
    ell = cfg.ells() if ell is None else ell
    C, err, lev, _ = O.cl_grid(ell, types, cfg.k_min, cfg.k_max, cfg.n_cheb, chi, wchi, R, wR, inp.P,
                               cfg.n_g, cfg.n_s, inp.Kchi, inp.Kchi2)
    assert err < 1e-9
    return C


TINY = [
    dict(),                                                            # 6 ell, 12 chi, 10 R, 24 nodes
    dict(n_ell=17, ell_max=90, n_chi=9, n_R=7, n_cheb=40, k_max=1.2),  # ragged everything
    dict(n_ell=3, ell_max=12, n_chi=5, n_R=3, n_cheb=2, k_max=0.3, n_g=1, n_s=3),
    dict(n_ell=9, ell_max=60, n_chi=7, n_R=6, n_cheb=32, k_max=0.8, n_g=3, n_s=1),  # MFMA projection
]


@pytest.fixture(scope="module", params=range(len(TINY)))
def tiny(request):
    cfg = W.tiny_config(**TINY[request.param])
    print("tiny config", request.param, cfg, flush=True)
    plan = B.plan_for_config(cfg, precisions=("fp64", "fp32", "bf16", "bf16x3"))
    inp = W.make_inputs(cfg, W.seed_for(9, request.param), plan.k_nodes, plan.chi, plan.R)
    Cor = _oracle(cfg, inp)
    yield cfg, plan, inp, Cor
    plan.close()


def test_tiny_fp64_matches_oracle(tiny):
    cfg, plan, inp, Cor = tiny
    C = _run(plan, inp, "fp64")
    e = g16_err(C, Cor, cfg.n_g, cfg.n_s)
    print("fp64 max err", e.max())
    assert e.max() <= 1e-6


@pytest.mark.parametrize("prec,p32,tol", [("fp32", True, 1e-3), ("bf16x3", True, 1e-3), ("bf16", True, 3e-2),
                                          ("fp32", False, 1e-3)])
def test_tiny_mixed_matches_oracle(tiny, prec, p32, tol):
    cfg, plan, inp, Cor = tiny
    C = _run(plan, inp, prec, p32=p32)
    e = g16_err(C, Cor, cfg.n_g, cfg.n_s)
    print(prec, "max err", e.max())
    assert e.max() <= tol


def test_basis_rows_match_oracle_integrals(tiny):
    """Ttilde_{n;l}(chi_a, R_b chi_a) of Eq. t_tilde = the oracle's k-integral with P = T_n."""
    cfg, plan, inp, _ = tiny
    rng = np.random.default_rng(3)
    for a, b in [(0, 0), (cfg.n_chi - 1, cfg.n_R - 1), (int(rng.integers(cfg.n_chi)), int(rng.integers(cfg.n_R)))]:
        T = plan.basis_point(a, b).reshape(3, plan.n_ell, plan.n_cheb)
        c1, c2 = plan.chi[a], plan.chi[a] * plan.R[b]
        coef = np.eye(plan.n_cheb)
        ref = np.stack([O.w_points(plan.ell, ALL, cfg.k_min, cfg.k_max, [c1], [c2], mode=O.P_CHEB,
                                   cheb_coef=coef[n], shared=True, M=max(64, 2 * plan.n_cheb))[:, :, 0]
                        for n in range(plan.n_cheb)], axis=-1)   # [3, n_ell, n_cheb]
        # rows of one type span many decades (ss at l = 2 vs l = 90); the two quadratures differ
        # by rounding of the oscillatory sum, so the bar is relative to the row plus a floor
        # relative to the whole type block
        row = np.abs(ref).max(axis=-1, keepdims=True)
        blk = np.abs(ref).max(axis=(1, 2), keepdims=True)
        bad = np.abs(T - ref) / (1e-9 * row + 1e-14 * blk)
        assert bad.max() <= 1.0, (a, b, np.unravel_index(bad.argmax(), bad.shape), bad.max())


def test_w_save_matches_oracle_w(tiny):
    """w_l(chi_a, R_b chi_a) of Eq. pmd at every grid point, FP64 path."""
    cfg, plan, inp, _ = tiny
    w = torch.zeros(len(plan.chi) * len(plan.R) * plan.rows_pad, dtype=torch.float64, device="cuda")
    _run(plan, inp, "fp64", w_save=w)
    wg = w.cpu().numpy().reshape(len(plan.chi), len(plan.R), plan.rows_pad)[:, :, :plan.rows]
    wg = wg.reshape(len(plan.chi) * len(plan.R), 3, plan.n_ell).transpose(1, 2, 0)
    c1 = np.repeat(plan.chi, len(plan.R))
    c2 = (plan.chi[:, None] * plan.R[None, :]).ravel()
    wo = O.w_points(plan.ell, ALL, cfg.k_min, cfg.k_max, c1, c2, nc=cfg.n_cheb,
                    P=inp.P.reshape(-1, cfg.n_cheb))
    scale = np.abs(wo).max(axis=-1, keepdims=True)
    assert np.all(np.abs(wg - wo) <= 1e-9 * scale)


def test_batch_invariance_and_subsets(tiny):
    """Each cosmology's result is bitwise the same alone and inside a batch; a types
    subset and an ell subset are bitwise slices of the full result."""
    cfg, plan, inp, _ = tiny
    inps = [inp] + [W.make_inputs(cfg, W.seed_for(9, 50 + i), plan.k_nodes, plan.chi, plan.R) for i in range(4)]
    P = _dev(np.stack([x.P for x in inps]))
    K1 = _dev(np.stack([x.Kchi for x in inps]))
    K2 = _dev(np.stack([x.Kchi2 for x in inps]))
    for prec in ("fp64", "fp32", "bf16x3"):
        Pp = P if prec == "fp64" else P.float()
        Cb = plan.forward(Pp, K1, K2, cfg.n_g, cfg.n_s, precision=prec).cpu().numpy()
        for i in range(len(inps)):
            # a copy: a view one cosmology into the batch need not be 16-byte aligned, as P must be
            Ci = plan.forward(Pp[i:i + 1].clone(), K1[i:i + 1].contiguous(), K2[i:i + 1].contiguous(),
                              cfg.n_g, cfg.n_s, precision=prec).cpu().numpy()
            assert np.array_equal(Ci[0], Cb[i]), prec
    full = plan.forward(P, K1, K2, cfg.n_g, cfg.n_s).cpu().numpy()
    sub_types = ("gs",) if cfg.n_g and cfg.n_s else ("gg",)
    Cs = plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, types=sub_types).cpu().numpy()
    pairs_all = W.pair_list(cfg.n_g, cfg.n_s)
    sel = [p for p, pr in enumerate(pairs_all) if pr[0] in sub_types]
    assert np.array_equal(Cs, full[:, sel])
    idx = np.arange(0, plan.n_ell, 2)
    Ce = plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, ell_idx=idx).cpu().numpy()
    assert np.array_equal(Ce, full[:, :, idx])


def test_forward_rejects_bad_arguments(tiny):
    cfg, plan, inp, _ = tiny
    P = _dev(inp.P[None])
    K1, K2 = _dev(inp.Kchi[None]), _dev(inp.Kchi2[None])
    with pytest.raises(B.BlastError) as e:
        plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, ell_idx=[1, 1])
    assert e.value.status == B.E_INVALID
    with pytest.raises(B.BlastError):
        plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, types=8)
    small = B.Plan(plan.ell, plan.chi, plan.w_chi, plan.R, plan.w_R, cfg.k_min, cfg.k_max, cfg.n_cheb,
                   precisions=("fp64",))
    with pytest.raises(B.BlastError):
        small.forward(P.float(), K1, K2, cfg.n_g, cfg.n_s, precision="fp32")   # not resident
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.BlastError):
        plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, workspace=ws)               # too small
    small.close()


def test_caller_workspace_gives_identical_result(tiny):
    cfg, plan, inp, _ = tiny
    nbytes = plan.workspace_bytes(2, "fp32", cfg.n_g + cfg.n_s)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    inps = [inp, W.make_inputs(cfg, W.seed_for(9, 77), plan.k_nodes, plan.chi, plan.R)]
    P = _dev(np.stack([x.P for x in inps]), torch.float32)
    K1 = _dev(np.stack([x.Kchi for x in inps]))
    K2 = _dev(np.stack([x.Kchi2 for x in inps]))
    a = plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, precision="fp32").cpu().numpy()
    b = plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, precision="fp32", workspace=ws).cpu().numpy()
    assert np.array_equal(a, b)


# ----------------------------------------------------------------------------- named configurations

def _golden(config):
    path = os.path.join(GOLDEN, "c%d_oracle.json" % config)
    if not os.path.exists(path):
        pytest.skip("no oracle golden for config %d" % config)
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("config", [1, 2])
def test_named_config_matches_oracle_golden(config):
    g = _golden(config)
    cfg = W.CONFIGS[config]
    print("config", config, "building plan", flush=True)
    t0 = time.time()
    plan = B.plan_for_config(cfg, precisions=("fp64", "fp32", "bf16x3", "bf16"))
    print("plan built in %.1fs (kq nodes %d)" % (time.time() - t0, plan.kq_nodes), flush=True)
    inp = W.make_inputs(cfg, g["seed"], plan.k_nodes, plan.chi, plan.R)
    assert abs(inp.cosmo.A - g["A"]) < 1e-9 * g["A"]
    Cor = np.array(g["C"])
    assert g["oracle_rel_change"] < 1e-9
    res = {}
    # bars of the library's stated accuracy (blast_hip.h): error ~ u * kappa, with kappa the
    # cancellation of the problem, largest for the gg cross spectra of separated bins at high ell.
    # BF16X3 (u ~ 2^-15) meets 1e-3 on the small grid only and stays within 2e-2 at the full
    # 3x2pt shapes (9.2e-3 measured, so kappa ~ 300 there); plain BF16 (u ~ 2^-7) is not an
    # accurate path: its stated bounds, 0.5 and 20, are u * kappa with that kappa and a factor
    # of 2-3 to spare (0.26 and 6.2 measured), and catch a regression or a non-finite result.
    x3_tol, b16_tol = (1e-3, 0.5) if config == 1 else (2e-2, 20.0)
    for prec, tol, p32 in (("fp64", 1e-6, False), ("fp32", 1e-3, True), ("bf16x3", x3_tol, True),
                           ("bf16", b16_tol, True)):
        C = _run(plan, inp, prec, p32=p32)
        e = g16_err(C, Cor, cfg.n_g, cfg.n_s)
        res[prec] = float(e.max())
        assert np.isfinite(C).all() and e.max() <= tol, (prec, e.max())
    print("config", config, "max errors", res, flush=True)
    plan.close()


@pytest.mark.parametrize("config", [1, 2])
def test_named_config_delta_chi2(config):
    """The paper's accuracy metric (Eq. dchi, LSST-like noise, f_sky = 0.4) of the FP32 path with
    the oracle golden as the benchmark: below the challenge's 0.2 (and reported without noise)."""
    from paper_2410_03632_amd import metrics as M
    g = _golden(config)
    cfg = W.CONFIGS[config]
    plan = B.plan_for_config(cfg, precisions=("fp64", "fp32"))
    try:
        inp = W.make_inputs(cfg, g["seed"], plan.k_nodes, plan.chi, plan.R)
        Cor = np.array(g["C"])
        pairs = W.pair_list(cfg.n_g, cfg.n_s)
        out = {}
        for prec in ("fp64", "fp32"):
            C = _run(plan, inp, prec, p32=prec == "fp32")
            out[prec] = (M.delta_chi2(C, Cor, plan.ell, cfg.n_g, cfg.n_s, pairs),
                         M.delta_chi2(C, Cor, plan.ell, cfg.n_g, cfg.n_s, pairs, N=np.zeros(cfg.n_g + cfg.n_s)))
        print("config", config, "Delta chi^2 (with noise, without):", out, flush=True)
        assert out["fp32"][0] < 0.2 and out["fp64"][0] < 1e-6
    finally:
        plan.close()


FUSED = [  # (n_g, n_s, n_cheb): weight groups NB = 4, 16 (rotated granules), 20 (five groups), 8;
    (2, 2, 24),     # and 2, 4, 6, 8 steps of 16 Chebyshev columns
    (10, 5, 40),
    (12, 6, 96),
    (3, 5, 128),
]


@pytest.mark.parametrize("n_g,n_s,n_cheb", FUSED)
@pytest.mark.parametrize("batch", [40, 70])
def test_fused_batch_matches_single_calls_and_oracle(n_g, n_s, n_cheb, batch):
    """From 32 cosmologies on, the mixed paths fuse the contraction with the R-quadrature (w stays
    in registers); a single cosmology takes the unfused kernels.  Every cosmology of a fused call
    must agree with its own single call, and the first with the oracle.  The two paths sum in
    different orders; each carries a rounding error of 1e-5..1e-4 of the spectra (FP32, BF16x3)
    against the oracle, so they may differ by a few times that, far inside the 1e-3 bar."""
    cfg = W.tiny_config(n_ell=7, ell_max=50, n_chi=10, n_R=9, n_cheb=n_cheb, k_max=0.6, n_g=n_g, n_s=n_s)
    print("fused case", n_g, n_s, n_cheb, batch, flush=True)
    plan = B.plan_for_config(cfg, precisions=("fp64", "fp32", "bf16", "bf16x3"))
    try:
        inps = [W.make_inputs(cfg, W.seed_for(12, i), plan.k_nodes, plan.chi, plan.R, vary=True) for i in range(batch)]
        P = _dev(np.stack([x.P for x in inps]), torch.float32)
        K1 = _dev(np.stack([x.Kchi for x in inps]))
        K2 = _dev(np.stack([x.Kchi2 for x in inps]))
        Cor = _oracle(cfg, inps[0])
        # plain BF16 (8-bit products) is a reported mode only: its error against the oracle grows
        # with the Chebyshev order (0.55 at 96 columns here), the same in both paths
        for prec, tol_single, tol_oracle in (("fp32", 3e-4, 1e-3), ("bf16x3", 4e-4, 1e-3), ("bf16", 1e-3, None)):
            Cb = plan.forward(P, K1, K2, n_g, n_s, precision=prec).cpu().numpy()
            worst = 0.0
            for i in list(range(0, batch, 7)) + [batch - 1]:
                Ci = plan.forward(P[i:i + 1].clone(), K1[i:i + 1].contiguous(), K2[i:i + 1].contiguous(), n_g,
                                  n_s, precision=prec).cpu().numpy()[0]
                worst = max(worst, g16_err(Cb[i], Ci, n_g, n_s).max())
            eo = g16_err(Cb[0], Cor, n_g, n_s).max()
            print(prec, "fused vs single", worst, "vs oracle", eo, flush=True)
            assert worst <= tol_single and (tol_oracle is None or eo <= tol_oracle), (prec, worst, eo)
    finally:
        plan.close()


@pytest.mark.parametrize("config", [1, 2])
def test_named_config_fused_batch_matches_oracle_golden(config):
    """The fused path (a batch of 32 copies of the golden cosmology) at the named shapes: config 1
    has 20 multipoles, so row tiles straddle the gg / gs / ss slots; config 2 has 96, so every
    tile holds one type and the R-sum keeps only that type's bins."""
    g = _golden(config)
    cfg = W.CONFIGS[config]
    plan = B.plan_for_config(cfg, precisions=("fp32",))
    try:
        inp = W.make_inputs(cfg, g["seed"], plan.k_nodes, plan.chi, plan.R)
        nb = 32
        P = _dev(np.repeat(inp.P[None], nb, axis=0), torch.float32)
        K1 = _dev(np.repeat(inp.Kchi[None], nb, axis=0))
        K2 = _dev(np.repeat(inp.Kchi2[None], nb, axis=0))
        C = plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, precision="fp32").cpu().numpy()
        Cor = np.array(g["C"])
        e = max(g16_err(C[i], Cor, cfg.n_g, cfg.n_s).max() for i in (0, nb - 1))
        print("config", config, "fused FP32 batch: max err", e, flush=True)
        assert e <= 1e-3
    finally:
        plan.close()
