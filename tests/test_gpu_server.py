"""GPU checks of the continuous-batching server (blast_server_*).

Requests with uneven bins and multipoles go through the server; each result must equal
the direct forward call for that request, and be bitwise the same whether the request
ran alone or mixed into a batch with others (per-cosmology arithmetic never mixes batch
entries)."""
import numpy as np
import pytest

from paper_2410_03632_amd import blast as B
from paper_2410_03632_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MAXG, MAXS = 4, 3


@pytest.fixture(scope="module")
def env():
    cfg = W.tiny_config(n_ell=24, ell_max=120, n_chi=16, n_R=12, n_cheb=32, k_max=0.8, n_g=MAXG, n_s=MAXS)
    plan = B.plan_for_config(cfg, precisions=("fp64", "fp32", "fp16x3"))
    chi, chi2 = plan.eval_points()
    Kchi, Kchi2 = W.kernels(W.bins_of(cfg), chi, chi2)
    rng = np.random.default_rng(12)
    reqs = []
    for i in range(24):
        cos = W.draw_cosmo(np.random.default_rng(W.seed_for(8, i)), vary=True)
        P = W.p_grid(plan.k_nodes, chi, chi2, cos)
        ng = int(rng.integers(0, MAXG + 1))
        ns = int(rng.integers(0 if ng else 1, MAXS + 1))
        nl = int(rng.integers(1, plan.n_ell + 1))
        idx = np.sort(rng.choice(plan.n_ell, nl, replace=False)).astype(np.int32)
        K1, K2 = W.request_kernels(Kchi, Kchi2, ng, ns, max_g=MAXG)
        reqs.append((P, ng, ns, idx, K1, K2))
    yield cfg, plan, reqs
    plan.close()


def _direct(plan, req, precision, pdt):
    P, ng, ns, idx, K1, K2 = req
    t = lambda x, d=torch.float64: torch.as_tensor(np.ascontiguousarray(x), dtype=d).cuda()
    C = plan.forward(t(P, pdt).unsqueeze(0).contiguous(), t(K1).unsqueeze(0).contiguous(),
                     t(K2).unsqueeze(0).contiguous(), ng, ns, precision=precision, ell_idx=idx)
    return C[0].cpu().numpy()


@pytest.mark.parametrize("precision,pdt,graphs", [("fp64", "fp64", True), ("fp32", "fp32", True),
                                                  ("fp32", "fp32", False), ("fp16x3", "fp32", True)])
def test_server_results_equal_direct_forward(env, precision, pdt, graphs):
    cfg, plan, reqs = env
    npdt = np.float64 if pdt == "fp64" else np.float32
    srv = B.Server(plan, precision=precision, p_dtype=pdt, batch=8, n_sets=2, max_g=MAXG, max_s=MAXS,
                   max_wait_ms=1.0, use_graphs=graphs)
    tickets = [srv.submit(np.ascontiguousarray(P, dtype=npdt), K1, K2, ng, ns, idx)
               for (P, ng, ns, idx, K1, K2) in reqs]
    outs = [srv.wait(t)[0] for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs) and st["rejected"] == 0
    assert st["p50_ms"] <= st["p99_ms"]
    tdt = torch.float64 if pdt == "fp64" else torch.float32
    for req, got in zip(reqs, outs):
        ref = _direct(plan, req, precision, tdt)
        assert got.shape == ref.shape
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max()), np.abs(got - ref).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16x3"])
def test_result_same_alone_and_in_the_mix(env, precision):
    cfg, plan, reqs = env
    pdt = np.float64 if precision == "fp64" else np.float32
    srv = B.Server(plan, precision=precision, p_dtype="fp64" if precision == "fp64" else "fp32", batch=8,
                   n_sets=2, max_g=MAXG, max_s=MAXS, max_wait_ms=5.0)
    X = reqs[3]
    P = np.ascontiguousarray(X[0], dtype=pdt)
    alone, _ = srv.wait(srv.submit(P, X[4], X[5], X[1], X[2], X[3]))
    alone = alone.copy()
    tk = []
    for i, (Pi, ng, ns, idx, K1, K2) in enumerate(reqs):
        tk.append(srv.submit(np.ascontiguousarray(Pi, dtype=pdt), K1, K2, ng, ns, idx))
        if i == 10:
            tx = srv.submit(P, X[4], X[5], X[1], X[2], X[3])
    mixed, _ = srv.wait(tx)
    for t in tk:
        srv.wait(t)
    st = srv.stats()
    srv.close()
    assert st["mean_fill"] > 1.0  # the mix really shared launches
    assert np.array_equal(alone, mixed)


def test_server_rejects_malformed_requests(env):
    cfg, plan, reqs = env
    srv = B.Server(plan, precision="fp32", p_dtype="fp32", batch=4, n_sets=1, max_g=MAXG, max_s=MAXS)
    P, ng, ns, idx, K1, K2 = reqs[0]
    P32 = np.ascontiguousarray(P, dtype=np.float32)
    Kg, Kg2 = W.request_kernels(*W.kernels(W.bins_of(cfg), *plan.eval_points()), MAXG, MAXS, max_g=MAXG)
    with pytest.raises(B.BlastError) as e:   # too many clustering bins
        srv.submit(P32, np.vstack([Kg, Kg[:1]]), np.concatenate([Kg2, Kg2[:1]]), MAXG + 1, MAXS, idx)
    assert e.value.status == B.E_INVALID
    with pytest.raises(B.BlastError):        # multipole indices not increasing
        srv.submit(P32, K1, K2, ng, ns, idx[::-1].copy() if len(idx) > 1 else np.array([5, 5], np.int32))
    with pytest.raises(B.BlastError):        # no bins
        srv.submit(P32, K1[:0], K2[:0], 0, 0, idx)
    assert srv.stats()["rejected"] == 3
    srv.close()
