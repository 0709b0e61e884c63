"""GPU checks of blast_cl_forward_noalloc, the forward for callers that cannot allocate: its
scratch is a fixed 64 MiB device array per GPU instead of plan-owned or caller memory.

It runs the same kernels in the same order as blast_cl_forward, so its spectra must equal the
forward's bit for bit.  Two calls in a row, the second smaller (fewer cosmologies, fewer bins,
a multipole subset), check that a call does not depend on what the previous one left in the
shared array.  Calls whose scratch exceeds the array, and calls that pass a workspace, are
refused before any work."""
import ctypes as C

import numpy as np
import pytest

from paper_2410_03632_amd import blast as B
from paper_2410_03632_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).cuda()


def _call_abi(plan, P, K1, K2, n_g, n_s, precision, ell_idx=None, workspace=None):
    """blast_cl_forward_noalloc called with ctypes on arguments the binding marshals."""
    args, keep, shape, _ = plan._prepare(P, K1, K2, n_g, n_s, precision, None, ell_idx, False)
    out = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
    args.C = out.data_ptr()
    if workspace is not None:
        args.workspace = workspace.data_ptr()
        args.workspace_bytes = workspace.numel()
    st = B.lib().blast_cl_forward_noalloc(plan.handle, C.byref(args),
                                          C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return st, out, keep


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16x3"])
@pytest.mark.parametrize("big", [5, 40])
def test_noalloc_equals_forward_twice_second_smaller(precision, big):
    """A batch of `big` cosmologies (40: the fused paths), then 2 cosmologies with 2 + 1 of the
    bins and 5 of the multipoles: both bitwise equal to blast_cl_forward on the same inputs."""
    cfg = W.tiny_config(n_ell=9, ell_max=60, n_chi=10, n_R=9, n_cheb=32, k_max=0.8, n_g=3, n_s=2)
    print("no-alloc", precision, big, flush=True)
    plan = B.plan_for_config(cfg, precisions=("fp64", "fp32", "fp16x3"))
    try:
        pdt = torch.float64 if precision == "fp64" else torch.float32
        inps = [W.make_inputs(cfg, W.seed_for(41, i), plan.k_nodes, plan.chi, plan.R, vary=True) for i in range(big)]
        P = _dev(np.stack([x.P for x in inps]), pdt)
        K1 = _dev(np.stack([x.Kchi for x in inps]))
        K2 = _dev(np.stack([x.Kchi2 for x in inps]))
        st, got, _ = _call_abi(plan, P, K1, K2, 3, 2, precision)
        assert st == B.OK, B.lib().blast_last_error()
        ref = plan.forward(P, K1, K2, 3, 2, precision=precision)
        torch.cuda.synchronize()
        assert torch.isfinite(got).all() and torch.equal(got, ref)
        # second call: 2 cosmologies, clustering bins 0-1 and shear bin 0, multipoles 1, 2, 4, 6, 8
        bsel = [0, 1, 3]
        idx = np.array([1, 2, 4, 6, 8], dtype=np.int32)
        P2 = P[3:5].clone()
        K1s, K2s = K1[3:5][:, bsel].contiguous(), K2[3:5][:, bsel].contiguous()
        st, got2, _ = _call_abi(plan, P2, K1s, K2s, 2, 1, precision, ell_idx=idx)
        assert st == B.OK, B.lib().blast_last_error()
        ref2 = plan.forward(P2, K1s, K2s, 2, 1, precision=precision, ell_idx=idx)
        torch.cuda.synchronize()
        assert torch.isfinite(got2).all() and torch.equal(got2, ref2)
        # the binding's wrapper of the same entry point
        out = torch.empty_like(ref2)
        plan.forward_noalloc(P2, K1s, K2s, 2, 1, out, precision=precision, ell_idx=idx)
        torch.cuda.synchronize()
        assert torch.equal(out, ref2)
    finally:
        plan.close()


def test_noalloc_full_3x2pt_fits_one_cosmology_and_refuses_more():
    """At the full 3x2pt shapes one cosmology fits the 64 MiB scratch on the FP32, FP16X3 and FP64
    paths (nodal P with 128 nodes keeps no coefficients; bitwise equal to blast_cl_forward); two
    cosmologies on FP64 and a batch of 8 on FP32 exceed it and are refused with
    BLAST_E_UNSUPPORTED before any launch; a workspace argument is refused with BLAST_E_INVALID."""
    cfg = W.CONFIGS[2]
    plan = B.plan_for_config(cfg, precisions=("fp64", "fp32", "fp16x3"))
    try:
        inp = W.make_inputs(cfg, W.seed_for(2, 0), plan.k_nodes, plan.chi, plan.R)
        for precision in ("fp32", "fp16x3"):
            P = _dev(inp.P[None], torch.float32)
            K1, K2 = _dev(inp.Kchi[None]), _dev(inp.Kchi2[None])
            st, got, _ = _call_abi(plan, P, K1, K2, cfg.n_g, cfg.n_s, precision)
            assert st == B.OK, B.lib().blast_last_error()
            ref = plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, precision=precision)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), precision
        P64, K1, K2 = _dev(inp.P[None]), _dev(inp.Kchi[None]), _dev(inp.Kchi2[None])
        st, got, _ = _call_abi(plan, P64, K1, K2, cfg.n_g, cfg.n_s, "fp64")
        assert st == B.OK, B.lib().blast_last_error()
        ref = plan.forward(P64, K1, K2, cfg.n_g, cfg.n_s, precision="fp64")
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        st, got, _ = _call_abi(plan, P64.expand(2, -1, -1, -1).contiguous(), K1.expand(2, -1, -1).contiguous(),
                               K2.expand(2, -1, -1, -1).contiguous(), cfg.n_g, cfg.n_s, "fp64")
        assert st == B.E_UNSUPPORTED and torch.isnan(got).all()
        P8 = _dev(inp.P[None], torch.float32).expand(8, -1, -1, -1).contiguous()
        K18 = _dev(inp.Kchi[None]).expand(8, -1, -1).contiguous()
        K28 = _dev(inp.Kchi2[None]).expand(8, -1, -1, -1).contiguous()
        st, got, _ = _call_abi(plan, P8, K18, K28, cfg.n_g, cfg.n_s, "fp32")
        assert st == B.E_UNSUPPORTED and torch.isnan(got).all()
        ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
        st, _, _ = _call_abi(plan, P8[:1].contiguous(), K18[:1].contiguous(), K28[:1].contiguous(), cfg.n_g,
                             cfg.n_s, "fp32", workspace=ws)
        assert st == B.E_INVALID
    finally:
        plan.close()
