"""GPU checks of the hand-written adjoint (blast_cl_backward) and its autograd wrapper.

C is linear in P (nodal values or Chebyshev coefficients), in K_chi and in K_chi2
separately, so for L = <G, C> central finite differences on the FP64 path are exact
up to rounding; the bar there is 1e-9 relative.  The gradient with respect to the
Chebyshev coefficients is also compared with the oracle: for one (chi_a, R_b) point
and one n, dL/dc_n = <G, dC> where dC comes from the oracle's k-integral of T_n at
that point and its own chi-R sum.
"""
import numpy as np
import pytest

import oracle as O
from paper_2410_03632_amd import blast as B
from paper_2410_03632_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ALL = ("gg", "gs", "ss")


def _dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).cuda()


@pytest.fixture(scope="module", params=[0, 1, 2])
def setup(request):
    # the third set has 18 bins: the kernels' 32-wide bin tiles
    kw = [dict(), dict(n_ell=11, ell_max=70, n_chi=9, n_R=7, n_cheb=32, k_max=0.9, n_g=3, n_s=2),
          dict(n_ell=5, ell_max=40, n_chi=8, n_R=6, n_cheb=24, k_max=0.6, n_g=12, n_s=6)][request.param]
    cfg = W.tiny_config(**kw)
    plan = B.plan_for_config(cfg, precisions=("fp64", "fp32"))
    inps = [W.make_inputs(cfg, W.seed_for(5, request.param * 10 + i), plan.k_nodes, plan.chi, plan.R)
            for i in range(3)]
    P = _dev(np.stack([x.P for x in inps]))
    K1 = _dev(np.stack([x.Kchi for x in inps]))
    K2 = _dev(np.stack([x.Kchi2 for x in inps]))
    yield cfg, plan, P, K1, K2
    plan.close()


def _loss(plan, cfg, P, K1, K2, G, precision="fp64", coef=False):
    C = plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, precision=precision, coef=coef)
    return float((C * G).sum())


def test_adjoint_matches_exact_finite_differences(setup):
    cfg, plan, P, K1, K2 = setup
    gen = torch.Generator(device="cpu").manual_seed(1)
    shape = (P.shape[0], B.n_pairs(cfg.n_g, cfg.n_s), plan.n_ell)
    G = torch.randn(shape, generator=gen, dtype=torch.float64).cuda()
    dP, dK, dK2 = plan.backward(P, K1, K2, cfg.n_g, cfg.n_s, G)
    for X, dX, name in ((P, dP, "P"), (K1, dK, "K_chi"), (K2, dK2, "K_chi2")):
        for trial in range(3):
            v = torch.randn(X.shape, generator=gen, dtype=torch.float64).cuda() * X.abs().mean()
            h = 1e-3
            args = {"P": P, "K_chi": K1, "K_chi2": K2}
            args[name] = (X + h * v).contiguous()
            Lp = _loss(plan, cfg, args["P"], args["K_chi"], args["K_chi2"], G)
            args[name] = (X - h * v).contiguous()
            Lm = _loss(plan, cfg, args["P"], args["K_chi"], args["K_chi2"], G)
            fd = (Lp - Lm) / (2 * h)
            an = float((dX * v).sum())
            assert abs(fd - an) <= 1e-9 * max(abs(fd), abs(an)) + 1e-300, (name, fd, an)


def test_fp32_adjoint_close_to_fp64(setup):
    cfg, plan, P, K1, K2 = setup
    gen = torch.Generator(device="cpu").manual_seed(2)
    shape = (P.shape[0], B.n_pairs(cfg.n_g, cfg.n_s), plan.n_ell)
    G = torch.randn(shape, generator=gen, dtype=torch.float64).cuda()
    r64 = plan.backward(P, K1, K2, cfg.n_g, cfg.n_s, G, precision="fp64")
    r32 = plan.backward(P.float(), K1, K2, cfg.n_g, cfg.n_s, G, precision="fp32")
    for name, a, b in zip(("P", "K_chi", "K_chi2"), r64, r32):
        a, b = a.double().cpu().numpy(), b.double().cpu().numpy()
        # element-wise, with a floor of 1e-3 of the largest gradient of the cosmology: a gradient
        # entry is a sum of terms of both signs, and the FP32 path's error is ~2^-23 times the sum
        # of their magnitudes, not of the (possibly cancelled) entry
        for i in range(a.shape[0]):
            floor = 1e-3 * np.abs(a[i]).max()
            e = float((np.abs(a[i] - b[i]) / np.maximum(np.abs(a[i]), floor)).max())
            print("FP32 vs FP64 adjoint", name, "cosmology", i, "max element-wise error %.2e" % e, flush=True)
            assert e < 1e-3, (name, i, e)


@pytest.mark.parametrize("precision,batch", [("fp32", 70), ("fp64", 40)])
def test_batched_adjoint_equals_calls_on_slices(precision, batch):
    """Batches past one cosmology tile (64 on FP32, 32 on FP64) with a ragged last tile: every
    adjoint kernel keeps each cosmology's sums to itself and in the same order whatever tile it
    falls in, so the batched gradients equal those of calls on slices bit for bit.  On FP64 the
    batched gradients are also checked against exact central differences (C is linear in each
    input) at 1e-9."""
    cfg = W.tiny_config(n_ell=9, ell_max=60, n_chi=8, n_R=7, n_cheb=32, k_max=0.8, n_g=3, n_s=2)
    print("batched adjoint", precision, batch, flush=True)
    plan = B.plan_for_config(cfg, precisions=("fp64", "fp32"))
    try:
        pdt = torch.float64 if precision == "fp64" else torch.float32
        inps = [W.make_inputs(cfg, W.seed_for(33, i), plan.k_nodes, plan.chi, plan.R, vary=True) for i in range(batch)]
        P = _dev(np.stack([x.P for x in inps]), pdt)
        K1 = _dev(np.stack([x.Kchi for x in inps]))
        K2 = _dev(np.stack([x.Kchi2 for x in inps]))
        gen = torch.Generator(device="cpu").manual_seed(7)
        G = torch.randn((batch, B.n_pairs(cfg.n_g, cfg.n_s), plan.n_ell), generator=gen, dtype=torch.float64).cuda()
        full = plan.backward(P, K1, K2, cfg.n_g, cfg.n_s, G, precision=precision)
        cuts = [0, 1, 30, 33, 64, batch - 5, batch]
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            if hi <= lo:
                continue
            sl = slice(lo, hi)
            part = plan.backward(P[sl].clone(), K1[sl].contiguous(), K2[sl].contiguous(), cfg.n_g, cfg.n_s,
                                 G[sl].contiguous(), precision=precision)
            for name, f, q in zip(("P", "K_chi", "K_chi2"), full, part):
                assert torch.equal(f[sl], q), (precision, name, lo, hi)
        if precision == "fp64":
            for X, dX, name in ((P, full[0], "P"), (K1, full[1], "K_chi"), (K2, full[2], "K_chi2")):
                v = torch.randn(X.shape, generator=gen, dtype=torch.float64).cuda() * X.abs().mean()
                h = 1e-3
                args = {"P": P, "K_chi": K1, "K_chi2": K2}
                args[name] = (X + h * v).contiguous()
                Lp = _loss(plan, cfg, args["P"], args["K_chi"], args["K_chi2"], G)
                args[name] = (X - h * v).contiguous()
                Lm = _loss(plan, cfg, args["P"], args["K_chi"], args["K_chi2"], G)
                fd, an = (Lp - Lm) / (2 * h), float((dX * v).sum())
                print("batch", batch, name, "fd", fd, "adjoint", an, flush=True)
                assert abs(fd - an) <= 1e-9 * max(abs(fd), abs(an)), (name, fd, an)
    finally:
        plan.close()


def test_adjoint_refuses_plans_whose_transpose_tile_exceeds_lds():
    """The FP64 transposed contraction keeps the dw rows of 32 cosmologies in LDS (8 bytes per row
    each): with 3 x 214 multipoles (rows padded to 656) that is more than 160 KB, so an FP64 call
    that asks for dP is refused before any launch, while the kernel-table gradients, which do not
    use that tile, are computed.  The FP32 path (4 bytes per row) takes this plan: its dP is checked
    against exact central differences of the FP64 forward (C is linear in P)."""
    ell = np.arange(2, 216, dtype=np.float64)
    chi, wchi = B.grid_chi_simpson(4, 500.0, 1500.0)
    R, wR = B.grid_R_fejer(2, 0.5)
    plan = B.Plan(ell, chi, wchi, R, wR, 1e-3, 0.3, 8, precisions=("fp64", "fp32"))
    try:
        assert plan.rows_pad >= 640
        gen = torch.Generator(device="cpu").manual_seed(3)
        P = (1.0 + torch.rand((1, 4, 2, 8), generator=gen, dtype=torch.float64)).cuda()
        K1 = torch.rand((1, 2, 4), generator=gen, dtype=torch.float64).cuda()
        K2 = torch.rand((1, 2, 4, 2), generator=gen, dtype=torch.float64).cuda()
        G = torch.randn((1, 3, len(ell)), generator=gen, dtype=torch.float64).cuda()
        with pytest.raises(B.BlastError) as e:
            plan.backward(P, K1, K2, 1, 1, G, precision="fp64")
        assert e.value.status == B.E_UNSUPPORTED, e.value
        _, dK, dK2 = plan.backward(P, K1, K2, 1, 1, G, precision="fp64", want=("K_chi", "K_chi2"))
        torch.cuda.synchronize()
        assert torch.isfinite(dK).all() and torch.isfinite(dK2).all()
        dP = plan.backward(P.float(), K1, K2, 1, 1, G, precision="fp32", want=("P",))[0].double()
        v = torch.randn(P.shape, generator=gen, dtype=torch.float64).cuda()
        h = 1e-3
        Lp = float((plan.forward((P + h * v).contiguous(), K1, K2, 1, 1) * G).sum())
        Lm = float((plan.forward((P - h * v).contiguous(), K1, K2, 1, 1) * G).sum())
        fd, an = (Lp - Lm) / (2 * h), float((dP * v).sum())
        print("FP32 dP at rows_pad", plan.rows_pad, "fd", fd, "adjoint", an, flush=True)
        assert abs(fd - an) <= 1e-4 * abs(fd)
    finally:
        plan.close()


def test_fp32_forward_keeping_w_on_the_fused_path():
    """From 32 cosmologies on, an FP32 forward that keeps w (and Y) for the adjoint runs the fused
    contraction + R-quadrature, whose kernel stores the w tiles as it makes them: its spectra equal
    those of the same call without w_save bit for bit, its w matches the FP64 path's w to FP32
    rounding (relative to each row's largest value), and the adjoint from the kept w and Y matches
    the adjoint that recomputes them (unfused, another summation order) to FP32 rounding."""
    cfg = W.tiny_config(n_ell=9, ell_max=60, n_chi=8, n_R=7, n_cheb=32, k_max=0.8, n_g=3, n_s=2)
    plan = B.plan_for_config(cfg, precisions=("fp64", "fp32"))
    try:
        nb = 40
        inps = [W.make_inputs(cfg, W.seed_for(34, i), plan.k_nodes, plan.chi, plan.R, vary=True) for i in range(nb)]
        P = _dev(np.stack([x.P for x in inps]))
        K1 = _dev(np.stack([x.Kchi for x in inps]))
        K2 = _dev(np.stack([x.Kchi2 for x in inps]))
        P32 = P.float()
        nw = nb * len(plan.chi) * len(plan.R) * plan.rows_pad
        w32 = torch.full((nw,), float("nan"), dtype=torch.float32, device="cuda")
        y32 = torch.empty(plan.y_numel(nb, 5), dtype=torch.float32, device="cuda")
        C_keep = plan.forward(P32, K1, K2, 3, 2, precision="fp32", w_save=w32, y_save=y32)
        C_plain = plan.forward(P32, K1, K2, 3, 2, precision="fp32")
        torch.cuda.synchronize()
        assert torch.equal(C_keep, C_plain)
        w64 = torch.zeros(nw, dtype=torch.float64, device="cuda")
        plan.forward(P, K1, K2, 3, 2, precision="fp64", w_save=w64)
        a = w64.cpu().numpy().reshape(-1, plan.rows_pad)[:, :plan.rows]
        b = w32.double().cpu().numpy().reshape(-1, plan.rows_pad)[:, :plan.rows]
        scale = np.abs(a).max(axis=1, keepdims=True)
        ew = float((np.abs(a - b) / scale).max())
        print("fused FP32 w vs FP64 w, max error per row scale", ew, flush=True)
        assert np.isfinite(b).all() and ew < 1e-5
        G = torch.randn(C_keep.shape, generator=torch.Generator(device="cpu").manual_seed(9), dtype=torch.float64).cuda()
        g_keep = plan.backward(P32, K1, K2, 3, 2, G, precision="fp32", w_save=w32, y_save=y32)
        g_new = plan.backward(P32, K1, K2, 3, 2, G, precision="fp32")
        for name, x, y in zip(("P", "K_chi", "K_chi2"), g_keep, g_new):
            x, y = x.double().cpu().numpy(), y.double().cpu().numpy()
            e = float((np.abs(x - y) / np.maximum(np.abs(y), 1e-3 * np.abs(y).max())).max())
            print("adjoint from kept w, Y vs recomputed:", name, e, flush=True)
            assert e < 1e-4, (name, e)
    finally:
        plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_backward_reads_w_and_y_only_when_needed(setup, precision):
    """dP alone needs neither w nor Y, and dK_chi with Y kept needs no w: such calls skip the
    recomputation of w and must give the same gradients, bit for bit, as the full call with w
    and Y kept (the same kernels on the same dY).  The autograd function keeps only what the
    adjoint will read and gives the library's gradients."""
    cfg, plan, P, K1, K2 = setup
    if precision == "fp32":
        P = P.float()
    wdt = torch.float64 if precision == "fp64" else torch.float32
    B_ = P.shape[0]
    w = torch.empty(B_ * len(plan.chi) * len(plan.R) * plan.rows_pad, dtype=wdt, device="cuda")
    y = torch.empty(plan.y_numel(B_, cfg.n_g + cfg.n_s), dtype=wdt, device="cuda")
    C = plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, precision=precision, w_save=w, y_save=y)
    G = torch.randn(C.shape, generator=torch.Generator(device="cpu").manual_seed(7), dtype=torch.float64).cuda()
    dP, dK, dK2 = plan.backward(P, K1, K2, cfg.n_g, cfg.n_s, G, precision=precision, w_save=w, y_save=y)
    dPa = plan.backward(P, K1, K2, cfg.n_g, cfg.n_s, G, precision=precision, want=("P",))[0]
    dPb, dKb = plan.backward(P, K1, K2, cfg.n_g, cfg.n_s, G, precision=precision, want=("P", "K_chi"),
                             y_save=y)[:2]
    torch.cuda.synchronize()
    assert torch.equal(dPa, dP) and torch.equal(dPb, dP) and torch.equal(dKb, dK)
    # autograd with only P differentiable: no w or Y kept, the same dP
    fn = B.cl_function()
    Pg = P.clone().requires_grad_(True)
    L = (fn.apply(plan, Pg, K1, K2, cfg.n_g, cfg.n_s, precision) * G).sum()
    L.backward()
    assert torch.equal(Pg.grad, dP)
    # only K_chi differentiable: Y kept, no w
    K1g = K1.clone().requires_grad_(True)
    L = (fn.apply(plan, P, K1g, K2, cfg.n_g, cfg.n_s, precision) * G).sum()
    L.backward()
    assert torch.equal(K1g.grad, dK)
    # only K_chi2 differentiable: w kept
    K2g = K2.clone().requires_grad_(True)
    L = (fn.apply(plan, P, K1, K2g, cfg.n_g, cfg.n_s, precision) * G).sum()
    L.backward()
    assert torch.equal(K2g.grad, dK2)
