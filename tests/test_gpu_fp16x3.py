"""GPU parity of the FP16X3 contraction: basis and coefficients split into FP16 hi + lo parts
(about 22 significant bits each) with a power-of-two scale per basis row and per coefficient row,
hi*hi + hi*lo + lo*hi on FP16 MFMA, FP32 accumulate; fused with the R-quadrature at every batch.

The bar is the mixed paths' 1e-3 (relative error of ``metrics.g16_err``) against the FP64 oracle,
at small grids and at the two named shapes (stored oracle goldens).  The row scales are checked
by exact scaling: P -> 2^k P must give C -> 2^k C bit for bit, because every scale is a power of
two.  Requests outside the fused path are refused."""
import dataclasses
import json
import os

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


def _oracle(plan, cfg, inp):
    C, err, _, _ = O.cl_grid(plan.ell, ALL, cfg.k_min, cfg.k_max, cfg.n_cheb, plan.chi, plan.w_chi, plan.R,
                             plan.w_R, inp.P, inp.n_g, inp.n_s, inp.Kchi, inp.Kchi2)
    assert err < 1e-9
    return C


CASES = [  # (n_g, n_s, n_cheb): weight groups NB = 4, 16, 20, 8; 1, 2, 3, 4 blocks of 32 columns
    (2, 2, 24),
    (10, 5, 40),
    (12, 6, 96),
    (3, 5, 128),
]


@pytest.mark.parametrize("n_g,n_s,n_cheb", CASES)
def test_fp16x3_matches_oracle_at_any_batch(n_g, n_s, n_cheb):
    """Batches of 1, 5 and 70 (FP16X3 is fused at every batch; 70 = one full tile of 64
    cosmologies and a ragged one) against the oracle, and every cosmology of the batched call
    against its own call in a small batch."""
    cfg = W.tiny_config(n_ell=7, ell_max=50, n_chi=10, n_R=9, n_cheb=n_cheb, k_max=0.6, n_g=n_g, n_s=n_s)
    print("fp16x3 case", n_g, n_s, n_cheb, flush=True)
    plan = B.plan_for_config(cfg, precisions=("fp64", "fp16x3"))
    try:
        inps = [W.make_inputs(cfg, W.seed_for(21, i), plan.k_nodes, plan.chi, plan.R, vary=True) for i in range(70)]
        P = _dev(np.stack([x.P for x in inps]), torch.float32)
        K1 = _dev(np.stack([x.Kchi for x in inps]))
        K2 = _dev(np.stack([x.Kchi2 for x in inps]))
        Cor = _oracle(plan, cfg, inps[0])
        Cb = plan.forward(P, K1, K2, n_g, n_s, precision="fp16x3").cpu().numpy()
        eo = g16_err(Cb[0], Cor, n_g, n_s).max()
        worst = 0.0
        for lo, nb in ((0, 1), (0, 5), (64, 6)):
            sl = slice(lo, lo + nb)
            Cs = plan.forward(P[sl].clone(), K1[sl].contiguous(), K2[sl].contiguous(), n_g, n_s,
                              precision="fp16x3").cpu().numpy()
            for i in range(nb):
                worst = max(worst, g16_err(Cs[i], Cb[lo + i], n_g, n_s).max())
        print("fp16x3 vs oracle", eo, "small batches vs 70", worst, flush=True)
        assert eo <= 1e-3 and worst <= 1e-6, (eo, worst)
    finally:
        plan.close()


def test_fp16x3_row_groups_with_a_short_last_group():
    """30 multipoles: 90 basis rows in 6 tiles of 16, two work-group row groups (4 and 2 tiles) of
    the wide fused kernel, with gg, gs and ss rows inside one group."""
    cfg = W.tiny_config(n_ell=30, ell_max=60, n_chi=10, n_R=9, n_cheb=64, k_max=0.6, n_g=4, n_s=3)
    plan = B.plan_for_config(cfg, precisions=("fp64", "fp16x3"))
    try:
        assert plan.rows_pad // 16 == 6
        inps = [W.make_inputs(cfg, W.seed_for(25, i), plan.k_nodes, plan.chi, plan.R, vary=True) for i in range(40)]
        P = _dev(np.stack([x.P for x in inps]), torch.float32)
        K1 = _dev(np.stack([x.Kchi for x in inps]))
        K2 = _dev(np.stack([x.Kchi2 for x in inps]))
        Cb = plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, precision="fp16x3").cpu().numpy()
        # the FP64 path on the FP64 inputs (P rounded to FP32 moves the cancelling cross spectra by ~1e-5)
        C64 = plan.forward(_dev(np.stack([inps[0].P, inps[39].P])), K1[[0, 39]].contiguous(),
                           K2[[0, 39]].contiguous(), cfg.n_g, cfg.n_s, precision="fp64").cpu().numpy()
        Cor = _oracle(plan, cfg, inps[0])
        e64 = g16_err(C64[0], Cor, cfg.n_g, cfg.n_s).max()
        eo = g16_err(Cb[0], Cor, cfg.n_g, cfg.n_s).max()
        el = g16_err(Cb[39], C64[1], cfg.n_g, cfg.n_s).max()
        print("30 ell: FP64 vs oracle", e64, "FP16X3 vs oracle", eo, "last cosmology vs FP64", el, flush=True)
        assert e64 <= 1e-6 and eo <= 1e-3 and el <= 1e-3
    finally:
        plan.close()


@pytest.mark.parametrize("config", [1, 2])
def test_fp16x3_named_config_matches_oracle_golden(config):
    """A batch of 32 copies of the golden cosmology at the named shapes."""
    g = json.load(open(os.path.join(GOLDEN, "c%d_oracle.json" % config)))
    cfg = W.CONFIGS[config]
    plan = B.plan_for_config(cfg, precisions=("fp16x3",))
    try:
        inp = W.make_inputs(cfg, g["seed"], plan.k_nodes, plan.chi, plan.R)
        nb = 32
        P = _dev(np.repeat(inp.P[None], nb, axis=0), torch.float32)
        K1 = _dev(np.repeat(inp.Kchi[None], nb, axis=0))
        K2 = _dev(np.repeat(inp.Kchi2[None], nb, axis=0))
        C = plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, precision="fp16x3").cpu().numpy()
        Cor = np.array(g["C"])
        e = max(g16_err(C[i], Cor, cfg.n_g, cfg.n_s).max() for i in (0, nb - 1))
        print("config", config, "FP16X3 batch: max err", e, flush=True)
        assert e <= 1e-3
    finally:
        plan.close()


def test_fp16x3_power_of_two_scaling_is_exact():
    """P -> 2^k P for k = +-40 (coefficient magnitudes far outside FP16's range): the row scales
    absorb the factor, so C scales exactly; a P row of zeros gives zero coefficients."""
    cfg = W.tiny_config(n_ell=6, ell_max=40, n_chi=8, n_R=6, n_cheb=32, k_max=0.4)
    plan = B.plan_for_config(cfg, precisions=("fp16x3",))
    try:
        inps = [W.make_inputs(cfg, W.seed_for(22, i), plan.k_nodes, plan.chi, plan.R, vary=True) for i in range(3)]
        P = _dev(np.stack([x.P for x in inps]), torch.float32)
        P[1, 2, 3].zero_()
        K1 = _dev(np.stack([x.Kchi for x in inps]))
        K2 = _dev(np.stack([x.Kchi2 for x in inps]))
        C0 = plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, precision="fp16x3").cpu().numpy()
        assert np.all(np.isfinite(C0))
        for k in (40, -40):
            Ck = plan.forward((P * 2.0 ** k).contiguous(), K1, K2, cfg.n_g, cfg.n_s, precision="fp16x3").cpu().numpy()
            assert np.array_equal(Ck, C0 * 2.0 ** k), k
    finally:
        plan.close()


@pytest.mark.parametrize("nb", [4, 70])
def test_fp16x3_coefficient_input(nb):
    """P given as Chebyshev coefficients (FP64) gives the nodal path's C to FP16X3 accuracy; 70
    cosmologies span two cosmology tiles of the fused kernel (one ragged) in the point-major
    coefficient layout that the coefficient input writes."""
    cfg = W.tiny_config(n_ell=6, ell_max=40, n_chi=8, n_R=6, n_cheb=40, k_max=0.4)
    plan = B.plan_for_config(cfg, precisions=("fp64", "fp16x3"))
    try:
        inps = [W.make_inputs(cfg, W.seed_for(23, i), plan.k_nodes, plan.chi, plan.R, vary=True) for i in range(nb)]
        Pn = np.stack([x.P for x in inps])
        N = plan.n_cheb
        _, xk = O.grid_k(N, cfg.k_min, cfg.k_max)
        T = np.cos(np.outer(np.arange(N), np.arccos(xk)))  # sum_n c_n T_n(x_j) = P_j
        c = np.linalg.solve(T.T, Pn.reshape(-1, N).T).T.reshape(Pn.shape)
        K1 = _dev(np.stack([x.Kchi for x in inps]))
        K2 = _dev(np.stack([x.Kchi2 for x in inps]))
        C64 = plan.forward(_dev(Pn), K1, K2, cfg.n_g, cfg.n_s, precision="fp64").cpu().numpy()
        Cc = plan.forward(_dev(c), K1, K2, cfg.n_g, cfg.n_s, precision="fp16x3", coef=True).cpu().numpy()
        e = max(g16_err(Cc[i], C64[i], cfg.n_g, cfg.n_s).max() for i in range(nb))
        print("fp16x3 coefficient input vs FP64 nodal", e, flush=True)
        assert e <= 1e-3
    finally:
        plan.close()


@pytest.mark.parametrize("n_cheb", [32, 64, 96, 128])
def test_fp16x3_nodal_basis_and_projection_agree(n_cheb):
    """FP32 nodal P runs the nodal basis (the DCT applied to the basis when the plan is made, P
    split in the kernel); FP64 nodal P takes the per-call projection into split coefficients.  Both
    against the oracle at the mixed paths' bar, at the first and last cosmology and at the one
    where the two paths differ most (they differ only by the rounding of their FP16 splits)."""
    cfg = W.tiny_config(n_ell=7, ell_max=60, n_chi=9, n_R=7, n_cheb=n_cheb, k_max=0.6, n_g=6, n_s=4)
    plan = B.plan_for_config(cfg, precisions=("fp16x3",))
    try:
        inps = [W.make_inputs(cfg, W.seed_for(26, i), plan.k_nodes, plan.chi, plan.R, vary=True) for i in range(67)]
        P64 = _dev(np.stack([x.P for x in inps]))
        K1 = _dev(np.stack([x.Kchi for x in inps]))
        K2 = _dev(np.stack([x.Kchi2 for x in inps]))
        Cn = plan.forward(P64.float().contiguous(), K1, K2, cfg.n_g, cfg.n_s, precision="fp16x3").cpu().numpy()
        Cp = plan.forward(P64, K1, K2, cfg.n_g, cfg.n_s, precision="fp16x3").cpu().numpy()
        d = [g16_err(Cn[i], Cp[i], cfg.n_g, cfg.n_s).max() for i in range(len(inps))]
        far = int(np.argmax(d))
        en, ep = 0.0, 0.0
        for i in sorted({0, len(inps) - 1, far}):
            Cor = _oracle(plan, cfg, inps[i])
            en = max(en, g16_err(Cn[i], Cor, cfg.n_g, cfg.n_s).max())
            ep = max(ep, g16_err(Cp[i], Cor, cfg.n_g, cfg.n_s).max())
        print("fp16x3 vs oracle: nodal", en, "projected", ep, "; largest difference", d[far], "at", far, flush=True)
        assert en <= 1e-3 and ep <= 1e-3, (en, ep)
    finally:
        plan.close()


@pytest.mark.parametrize("n_cheb,n_g,n_s", [(20, 6, 4), (20, 12, 6), (36, 3, 5), (68, 2, 2), (100, 10, 5)])
def test_fp16x3_fp32_nodal_p_with_n_cheb_a_multiple_of_four(n_cheb, n_g, n_s):
    """FP32 nodal P needs whole 16-byte granules per row (n_cheb % 4 == 0), not the projection's
    n_cheb % 8 == 0: the k nodes past n_cheb repeat the last granule against zero basis columns.
    With up to 16 bins the fused kernel splits P itself, with 17 to 20 P is split into coefficient
    rows first.  One to four blocks of 32 columns (20, 36, 68, 100 nodes).  Against the oracle at
    the mixed paths' bar, batch 1 and a batch of 70."""
    cfg = W.tiny_config(n_ell=6, ell_max=50, n_chi=8, n_R=6, n_cheb=n_cheb, k_max=0.5, n_g=n_g, n_s=n_s)
    plan = B.plan_for_config(cfg, precisions=("fp16x3",))
    try:
        inps = [W.make_inputs(cfg, W.seed_for(27, i), plan.k_nodes, plan.chi, plan.R, vary=True) for i in range(70)]
        P = _dev(np.stack([x.P for x in inps]), torch.float32)
        K1 = _dev(np.stack([x.Kchi for x in inps]))
        K2 = _dev(np.stack([x.Kchi2 for x in inps]))
        print("fp16x3 fp32 nodal P", n_cheb, n_g, n_s, flush=True)
        Cb = plan.forward(P, K1, K2, n_g, n_s, precision="fp16x3").cpu().numpy()
        C1 = plan.forward(P[-1:].contiguous(), K1[-1:].contiguous(), K2[-1:].contiguous(), n_g, n_s,
                          precision="fp16x3").cpu().numpy()
        e = 0.0
        for i in (0, 33, 69):
            # the oracle on the FP32-rounded P the kernel reads
            inp = dataclasses.replace(inps[i], P=inps[i].P.astype(np.float32).astype(np.float64))
            Cor = _oracle(plan, cfg, inp)
            e = max(e, g16_err(Cb[i], Cor, n_g, n_s).max())
            if i == 69:
                e = max(e, g16_err(C1[0], Cor, n_g, n_s).max())
        print("fp16x3 fp32 nodal P vs oracle", e, flush=True)
        assert e <= 1e-3
    finally:
        plan.close()


def test_fp16x3_refuses_requests_outside_the_fused_path():
    cfg = W.tiny_config(n_ell=4, ell_max=30, n_chi=6, n_R=5, n_cheb=22, k_max=0.4, n_g=12, n_s=9)
    plan = B.plan_for_config(cfg, precisions=("fp16x3",))
    try:
        inp = W.make_inputs(cfg, W.seed_for(24), plan.k_nodes, plan.chi, plan.R)
        P = _dev(inp.P[None], torch.float32)
        K1, K2 = _dev(inp.Kchi[None]), _dev(inp.Kchi2[None])
        # 21 bins
        with pytest.raises(B.BlastError) as e:
            plan.forward(P, K1, K2, 12, 9, precision="fp16x3")
        assert e.value.status == B.E_UNSUPPORTED
        # n_cheb = 22 is neither a multiple of 8 (FP64 nodal P) nor of 4 (FP32 nodal P); 10 bins
        # would otherwise be fine
        for Pd in (P, _dev(inp.P[None])):
            with pytest.raises(B.BlastError) as e:
                plan.forward(Pd, K1[:, :10].contiguous(), K2[:, :10].contiguous(), 6, 4, precision="fp16x3")
            assert e.value.status == B.E_UNSUPPORTED
        # w cannot be kept
        w = torch.empty(len(plan.chi) * len(plan.R) * plan.rows_pad, dtype=torch.float32, device="cuda")
        with pytest.raises(B.BlastError) as e:
            plan.forward(P, K1[:, :10].contiguous(), K2[:, :10].contiguous(), 6, 4, precision="fp16x3", w_save=w)
        assert e.value.status == B.E_UNSUPPORTED
        # the adjoint runs in FP64 or FP32
        dC = torch.zeros((1, 55, cfg.n_ell), dtype=torch.float64, device="cuda")
        with pytest.raises(B.BlastError) as e:
            plan.backward(P, K1[:, :10].contiguous(), K2[:, :10].contiguous(), 6, 4, dC, precision="fp16x3")
        assert e.value.status == B.E_UNSUPPORTED
    finally:
        plan.close()
