"""GPU parity of the FP64 fused contraction and R-quadrature: batches of 32 or more with at most 16
bins and no w_save run the contraction on FP64 MFMA with w kept in registers, an FP64 weights table
and Y accumulated in FP64.

Bars: against the oracle, the FP64 path's 1e-6 (relative error of ``metrics.g16_err``); against the
unfused FP64 path (the same call with w_save, which keeps w in memory and sums it in a separate
kernel) 1e-11, since the two differ only in the order of FP64 sums."""
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


CASES = [  # (n_g, n_s, n_cheb, n_ell): bins -> weight width, n_cheb -> stages, n_ell -> row tiles
    (2, 2, 24, 7),     # 4 bins; 32 columns (one stage of 32); 21 rows -> one group of 2 tiles
    (5, 3, 64, 5),     # 8 bins; 64 columns (one stage of 64); 15 rows -> a group with one tile
    (8, 4, 96, 7),     # 12 bins; 96 columns (three stages of 32)
    (10, 5, 128, 11),  # 15 bins (16 wide); 128 columns (two stages of 64); 33 rows -> groups of 2 and 1
]


@pytest.mark.parametrize("n_g,n_s,n_cheb,n_ell", CASES)
def test_fp64_fused_matches_unfused_and_oracle(n_g, n_s, n_cheb, n_ell):
    """Batch 70 (one full tile of 64 cosmologies and a ragged one of 6): every cosmology against
    the unfused FP64 path, the first and the last against the oracle; a batch of 31 (below the
    fused path's minimum) gives the same result as its cosmologies in the batch of 70."""
    cfg = W.tiny_config(n_ell=n_ell, ell_max=60, n_chi=10, n_R=9, n_cheb=n_cheb, k_max=0.6, n_g=n_g, n_s=n_s)
    print("fp64 fused case", n_g, n_s, n_cheb, n_ell, flush=True)
    plan = B.plan_for_config(cfg, precisions=("fp64",))
    try:
        nb = 70
        inps = [W.make_inputs(cfg, W.seed_for(31, i), plan.k_nodes, plan.chi, plan.R, vary=True) for i in range(nb)]
        P = _dev(np.stack([x.P for x in inps]))
        K1 = _dev(np.stack([x.Kchi for x in inps]))
        K2 = _dev(np.stack([x.Kchi2 for x in inps]))
        Cf = plan.forward(P, K1, K2, n_g, n_s, precision="fp64").cpu().numpy()
        w = torch.zeros(nb * len(plan.chi) * len(plan.R) * plan.rows_pad, dtype=torch.float64, device="cuda")
        Cu = plan.forward(P, K1, K2, n_g, n_s, precision="fp64", w_save=w).cpu().numpy()
        eu = max(g16_err(Cf[i], Cu[i], n_g, n_s).max() for i in range(nb))
        eo = 0.0
        for i in (0, nb - 1):
            Cor, err, _, _ = O.cl_grid(plan.ell, ALL, cfg.k_min, cfg.k_max, cfg.n_cheb, plan.chi, plan.w_chi, plan.R,
                                       plan.w_R, inps[i].P, n_g, n_s, inps[i].Kchi, inps[i].Kchi2)
            assert err < 1e-9
            eo = max(eo, g16_err(Cf[i], Cor, n_g, n_s).max())
        sl = slice(39, 70)
        Cs = plan.forward(P[sl].clone(), K1[sl].contiguous(), K2[sl].contiguous(), n_g, n_s,
                          precision="fp64").cpu().numpy()
        es = max(g16_err(Cs[i], Cf[39 + i], n_g, n_s).max() for i in range(31))
        print("fused vs unfused", eu, "vs oracle", eo, "batch 31 vs 70", es, flush=True)
        assert eu <= 1e-11 and eo <= 1e-6 and es <= 1e-11, (eu, eo, es)
    finally:
        plan.close()


@pytest.mark.parametrize("config", [1, 2])
def test_fp64_fused_named_config_matches_oracle_golden(config):
    """A batch of 32 copies of the golden cosmology through the fused FP64 kernel at both named
    shapes: 4 bins, 64 Chebyshev terms, 20 multipoles (row tiles that straddle the type slots),
    and the full 3x2pt workload (15 bins, 128 terms, 96 multipoles: 288 rows in 18 tiles, two
    stages of 64 columns), which is the shape the FP64 line of the benchmark times.  Every
    element of the first and the last copy against the oracle, and all copies bitwise equal
    (per-cosmology arithmetic never mixes batch entries)."""
    g = json.load(open(os.path.join(GOLDEN, "c%d_oracle.json" % config)))
    cfg = W.CONFIGS[config]
    print("FP64 fused, config", config, flush=True)
    plan = B.plan_for_config(cfg, precisions=("fp64",))
    try:
        inp = W.make_inputs(cfg, g["seed"], plan.k_nodes, plan.chi, plan.R)
        nb = 32
        P = _dev(inp.P[None]).expand(nb, -1, -1, -1).contiguous()
        K1 = _dev(inp.Kchi[None]).expand(nb, -1, -1).contiguous()
        K2 = _dev(inp.Kchi2[None]).expand(nb, -1, -1, -1).contiguous()
        C = plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, precision="fp64").cpu().numpy()
        Cor = np.array(g["C"])
        e = max(g16_err(C[i], Cor, cfg.n_g, cfg.n_s).max() for i in (0, nb - 1))
        print("config", config, "FP64 fused batch: max err", e, flush=True)
        assert np.isfinite(C).all() and e <= 1e-6
        assert all(np.array_equal(C[i], C[0]) for i in range(1, nb))
    finally:
        plan.close()


def test_fp64_coefficient_input_on_the_fused_path():
    """P given as Chebyshev coefficients at batch 32 matches the nodal input to FP64 rounding."""
    cfg = W.tiny_config(n_ell=6, ell_max=40, n_chi=8, n_R=6, n_cheb=40, k_max=0.4)
    plan = B.plan_for_config(cfg, precisions=("fp64",))
    try:
        nb = 32
        inps = [W.make_inputs(cfg, W.seed_for(32, i), plan.k_nodes, plan.chi, plan.R, vary=True) for i in range(nb)]
        Pn = np.stack([x.P for x in inps])
        N = plan.n_cheb
        _, xk = O.grid_k(N, cfg.k_min, cfg.k_max)
        T = np.cos(np.outer(np.arange(N), np.arccos(xk)))  # sum_n c_n T_n(x_j) = P_j
        c = np.linalg.solve(T.T, Pn.reshape(-1, N).T).T.reshape(Pn.shape)
        K1 = _dev(np.stack([x.Kchi for x in inps]))
        K2 = _dev(np.stack([x.Kchi2 for x in inps]))
        Cn = plan.forward(_dev(Pn), K1, K2, cfg.n_g, cfg.n_s, precision="fp64").cpu().numpy()
        Cc = plan.forward(_dev(c), K1, K2, cfg.n_g, cfg.n_s, precision="fp64", coef=True).cpu().numpy()
        e = max(g16_err(Cc[i], Cn[i], cfg.n_g, cfg.n_s).max() for i in range(nb))
        print("FP64 fused: coefficient input vs nodal", e, flush=True)
        assert e <= 1e-9
    finally:
        plan.close()
