"""GPU parity at the benchmark's own launch: the full 3x2pt shapes (10 + 5 bins, 96 ell, 256 chi,
96 R, 128 Chebyshev nodes) at a batch of 256 cosmologies, the grid ``bench.py`` times (four
cosmology tiles of 64, five row groups, every chi node).  The batch holds the stored oracle
cosmology (Eq. final_cls evaluated by the FP64 oracle, ``tests/golden/c2_oracle.json``) at
several places (the same kernel tables everywhere), the other places other seeded cosmologies;
the stored copies are compared element by element at each path's bar (1e-3 for the mixed paths,
1e-6 for FP64), and every output is checked finite.  The gradient step is checked at the same
launch against the FP64 adjoint."""
import json
import os

import numpy as np
import pytest

from paper_2410_03632_amd import blast as B
from paper_2410_03632_amd import workloads as W
from _util import g16_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SLOTS = (0, 63, 64, 191, 255)  # first and last of a tile, tiles 0, 1, 2, 3


@pytest.fixture(scope="module")
def full():
    g = json.load(open(os.path.join(GOLDEN, "c2_oracle.json")))
    cfg = W.CONFIGS[2]
    plan = B.plan_for_config(cfg, precisions=("fp64", "fp32", "fp16x3"))
    chi, chi2 = plan.eval_points()
    inp = W.make_inputs(cfg, g["seed"], plan.k_nodes, plan.chi, plan.R)
    others = [torch.as_tensor(W.p_grid(plan.k_nodes, chi, chi2, W.draw_cosmo(np.random.default_rng(W.seed_for(2, i)))))
              for i in range(1, 4)]
    yield cfg, plan, inp, others, np.array(g["C"])
    plan.close()


@pytest.mark.parametrize("prec,bar", [("fp16x3", 1e-3), ("fp32", 1e-3), ("fp64", 1e-6)])
def test_benchmark_launch_matches_the_stored_oracle_values(full, prec, bar):
    cfg, plan, inp, others, Cor = full
    nb = 256
    dt = torch.float64 if prec == "fp64" else torch.float32
    P = torch.empty((nb, cfg.n_chi, cfg.n_R, cfg.n_cheb), dtype=dt, device="cuda")
    gold = torch.as_tensor(inp.P, dtype=dt, device="cuda")
    oth = [o.to(device="cuda", dtype=dt) for o in others]
    for i in range(nb):
        P[i] = gold if i in SLOTS else oth[i % 3]
    K1 = torch.as_tensor(inp.Kchi, device="cuda").unsqueeze(0).expand(nb, -1, -1).contiguous()
    K2 = torch.as_tensor(inp.Kchi2, device="cuda").unsqueeze(0).expand(nb, -1, -1, -1).contiguous()
    print("full batch", prec, flush=True)
    C = plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, precision=prec)
    assert torch.isfinite(C).all()
    C = C.cpu().numpy()
    # FP32 P: the stored values are the oracle's for the FP64 P, whose FP32 rounding (6e-8) is far
    # below the bar
    e = max(g16_err(C[i], Cor, cfg.n_g, cfg.n_s).max() for i in SLOTS)
    # the copies of one cosmology agree with each other to the path's rounding
    d = max(g16_err(C[i], C[0], cfg.n_g, cfg.n_s).max() for i in SLOTS)
    print(prec, "batch 256 vs oracle", e, "copies", d, flush=True)
    assert e <= bar and d <= bar, (e, d)


def test_gradient_at_the_benchmark_launch(full):
    """The gradient step ``bench.py`` times (FP32: a forward keeping w and Y, then the adjoint to
    dP, dK_chi and dK_chi2) at batch 256 on the full shapes, against the FP64 adjoint of the
    stored cosmology alone, element by element with a floor of 1e-3 of the cosmology's largest
    gradient (an entry is a sum of terms of both signs, and FP32 rounds the sum of their
    magnitudes).  The adjoint to dP alone (a forward keeping nothing) gives the same dP bit for
    bit."""
    cfg, plan, inp, others, _ = full
    nb = 256
    P = torch.empty((nb, cfg.n_chi, cfg.n_R, cfg.n_cheb), dtype=torch.float32, device="cuda")
    gold = torch.as_tensor(inp.P, dtype=torch.float32, device="cuda")
    oth = [o.to(device="cuda", dtype=torch.float32) for o in others]
    for i in range(nb):
        P[i] = gold if i in SLOTS else oth[i % 3]
    K1 = torch.as_tensor(inp.Kchi, device="cuda").unsqueeze(0).expand(nb, -1, -1).contiguous()
    K2 = torch.as_tensor(inp.Kchi2, device="cuda").unsqueeze(0).expand(nb, -1, -1, -1).contiguous()
    shape = (nb, B.n_pairs(cfg.n_g, cfg.n_s), plan.n_ell)
    g1 = torch.randn(shape[1:], generator=torch.Generator(device="cpu").manual_seed(5), dtype=torch.float64)
    G = g1.cuda().unsqueeze(0).expand(shape).contiguous()
    w = torch.empty(nb * cfg.n_chi * cfg.n_R * plan.rows_pad, dtype=torch.float32, device="cuda")
    y = torch.empty(plan.y_numel(nb, cfg.n_g + cfg.n_s), dtype=torch.float32, device="cuda")
    print("full batch gradient", flush=True)
    plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, precision="fp32", w_save=w, y_save=y)
    r32 = plan.backward(P, K1, K2, cfg.n_g, cfg.n_s, G, precision="fp32", w_save=w, y_save=y)
    dp_only = plan.backward(P, K1, K2, cfg.n_g, cfg.n_s, G, precision="fp32", want=("P",))[0]
    assert torch.equal(dp_only, r32[0])
    P64 = torch.as_tensor(inp.P.astype(np.float32).astype(np.float64)[None], device="cuda")
    r64 = plan.backward(P64, K1[:1].contiguous(), K2[:1].contiguous(), cfg.n_g, cfg.n_s, G[:1].contiguous(),
                        precision="fp64")
    for name, a, b in zip(("P", "K_chi", "K_chi2"), r64, r32):
        assert torch.isfinite(b).all(), name
        a = a[0].double().cpu().numpy()
        floor = 1e-3 * np.abs(a).max()
        for i in SLOTS:
            e = float((np.abs(a - b[i].double().cpu().numpy()) / np.maximum(np.abs(a), floor)).max())
            print("batch 256 FP32 adjoint vs FP64", name, "place", i, "max element-wise error %.2e" % e, flush=True)
            assert e < 1e-3, (name, i, e)
