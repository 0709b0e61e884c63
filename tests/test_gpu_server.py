"""GPU checks of the continuous-batching server (blast_server_*).

Requests with uneven bins and multipoles go through the server; each result must equal the
direct forward call for that request and the FP64 oracle within each path's bar, and be the
same whether the request ran alone or mixed into a batch with others (per-cosmology
arithmetic never mixes batch entries).  Cancellation, polling, admission against the memory
budget and two sets in flight at once are checked too."""
import numpy as np
import pytest

import oracle as O
from paper_2410_03632_amd import blast as B
from paper_2410_03632_amd import workloads as W
from _util import g16_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MAXG, MAXS = 4, 3
ALL = ("gg", "gs", "ss")


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


# tolerance of "the same alone and in a mix": a mix can put a request in a larger bin bucket
# (more zero-kernel bins), which may change the fused kernels' R-sum width but no sum of the
# request's own numbers; the bars are far below each path's accuracy bar
MIX_TOL = {"fp64": 1e-12, "fp32": 1e-6, "fp16x3": 1e-6}


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16x3"])
def test_result_same_alone_and_in_the_mix(env, precision):
    cfg, plan, reqs = env
    pdt = np.float64 if precision == "fp64" else np.float32
    srv = B.Server(plan, precision=precision, p_dtype="fp64" if precision == "fp64" else "fp32", batch=8,
                   n_sets=2, max_g=MAXG, max_s=MAXS, max_wait_ms=5.0)
    for X in (reqs[3], reqs[5]):
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
        e = float(g16_err(mixed, alone, X[1], X[2]).max()) if mixed.size else 0.0
        print(precision, "bins", X[1], X[2], "alone vs mixed", e, "bitwise", np.array_equal(alone, mixed), flush=True)
        assert e <= MIX_TOL[precision]
    st = srv.stats()
    srv.close()
    assert st["mean_fill"] > 1.0  # the mix really shared launches


# the oracle's spectra of a few requests (their own bins, every plan multipole), computed once
@pytest.fixture(scope="module")
def oracle_of(env):
    cfg, plan, reqs = env
    chi, wchi = O.grid_chi(cfg.n_chi, cfg.chi_min, cfg.chi_max)
    R, wR = O.grid_R(cfg.n_R, cfg.R_min)
    out = {}
    for k in (0, 1, 2, 7, 13, 21):
        P, ng, ns, idx, K1, K2 = reqs[k]
        Cor, err, _, _ = O.cl_grid(plan.ell, ALL, cfg.k_min, cfg.k_max, cfg.n_cheb, chi, wchi, R, wR, P, ng, ns, K1,
                                   K2)
        assert err < 1e-9
        out[k] = Cor[:, idx]
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16x3"])
def test_server_results_match_oracle(env, oracle_of, precision):
    """Server results of requests with uneven bins (0-4 clustering, 0-3 shear) and multipole
    subsets, mixed into shared launches in padded bin buckets, element by element against the
    FP64 oracle on each request's own bins: the padded layout and the pair / multipole pick-out
    are server-only code that no direct call reaches."""
    cfg, plan, reqs = env
    pdt = np.float64 if precision == "fp64" else np.float32
    srv = B.Server(plan, precision=precision, p_dtype="fp64" if precision == "fp64" else "fp32", batch=8,
                   n_sets=2, max_g=MAXG, max_s=MAXS, max_wait_ms=2.0)
    tk = {k: srv.submit(np.ascontiguousarray(P, dtype=pdt), K1, K2, ng, ns, idx)
          for k, (P, ng, ns, idx, K1, K2) in enumerate(reqs)}
    outs = {k: srv.wait(t)[0] for k, t in tk.items()}
    st = srv.stats()
    srv.close()
    assert st["mean_fill"] > 1.0
    bar = 1e-6 if precision == "fp64" else 1e-3
    for k, Cor in oracle_of.items():
        P, ng, ns, idx, K1, K2 = reqs[k]
        e = float(g16_err(outs[k], Cor, ng, ns).max())
        print(precision, "request", k, "bins", ng, ns, "ell", len(idx), "max err vs oracle", e, flush=True)
        assert outs[k].shape == Cor.shape and e <= bar


def test_admission_by_memory(env):
    """A server whose arena holds one request without clustering bins but not one with the largest
    bucket refuses the latter with BLAST_E_OOM at submit and serves the former; one whose arena
    holds two small requests never launches more than two."""
    cfg, plan, reqs = env
    probe = B.Server(plan, precision="fp32", p_dtype="fp32", batch=8, n_sets=1, max_g=MAXG, max_s=MAXS)
    small1, _ = probe.footprint(0, MAXS, 1)
    small2, _ = probe.footprint(0, MAXS, 2)
    big1, _ = probe.footprint(MAXG, MAXS, 1)
    probe.close()
    assert small1 < big1
    small = [r for r in reqs if r[1] == 0]
    big = [r for r in reqs if r[1] > 0]
    assert small and big
    srv = B.Server(plan, precision="fp32", p_dtype="fp32", batch=8, n_sets=1, max_g=MAXG, max_s=MAXS,
                   hbm_budget=small1)
    P, ng, ns, idx, K1, K2 = big[0]
    with pytest.raises(B.BlastError) as e:
        srv.submit(np.ascontiguousarray(P, dtype=np.float32), K1, K2, ng, ns, idx)
    assert e.value.status == B.E_OOM
    P, ng, ns, idx, K1, K2 = small[0]
    got, _ = srv.wait(srv.submit(np.ascontiguousarray(P, dtype=np.float32), K1, K2, ng, ns, idx))
    srv.close()
    ref = _direct(plan, small[0], "fp32", torch.float32)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    srv = B.Server(plan, precision="fp32", p_dtype="fp32", batch=8, n_sets=1, max_g=MAXG, max_s=MAXS,
                   hbm_budget=small2, max_wait_ms=50.0)
    tk = [srv.submit(np.ascontiguousarray(r[0], dtype=np.float32), r[4], r[5], r[1], r[2], r[3]) for r in small * 3]
    for t in tk:
        srv.wait(t)
    st = srv.stats()
    srv.close()
    print("two-request arena: launches", st["launches"], "mean fill", st["mean_fill"], flush=True)
    assert st["completed"] == len(tk) and st["launches"] >= (len(tk) + 1) // 2 and st["mean_fill"] <= 2.0


@pytest.fixture(scope="module")
def big():
    """The full 3x2pt grid (a launch keeps the device busy for milliseconds) with one request
    shape: 2 clustering + 1 shear bins, every 5th multipole."""
    cfg = W.CONFIGS[2]
    plan = B.plan_for_config(cfg, precisions=("fp32",))
    chi, chi2 = plan.eval_points()
    Kchi, Kchi2 = W.kernels(W.bins_of(cfg), chi, chi2)
    K1, K2 = Kchi[[0, 1, 10]].copy(), Kchi2[[0, 1, 10]].copy()
    P = np.ascontiguousarray(W.p_grid(plan.k_nodes, chi, chi2, W.draw_cosmo(np.random.default_rng(3))),
                             dtype=np.float32)
    idx = np.arange(0, plan.n_ell, 5, dtype=np.int32)
    yield plan, P, K1, K2, idx
    plan.close()


def test_two_sets_in_flight(big):
    """With two sets of one slot and a burst of requests, the second set is launched while the
    first still runs; every request gets the same spectra."""
    plan, P, K1, K2, idx = big
    srv = B.Server(plan, precision="fp32", p_dtype="fp32", batch=1, n_sets=2, max_g=2, max_s=1, max_wait_ms=0.0)
    tk = [srv.submit(P, K1, K2, 2, 1, idx) for _ in range(6)]
    outs = [srv.wait(t)[0] for t in tk]
    st = srv.stats()
    srv.close()
    print("sets in flight at most", st["max_sets_in_flight"], "launches", st["launches"], flush=True)
    assert st["n_sets"] == 2 and st["max_sets_in_flight"] == 2
    assert all(np.array_equal(o, outs[0]) for o in outs)


def test_cancel_and_poll(big):
    """With the one set busy (each launch takes milliseconds), a queued request is cancelled: wait
    reports BLAST_E_CANCELLED, the others complete with the spectra of a direct call; cancelling a
    finished ticket is refused; poll returns None until its ticket completes."""
    plan, P, K1, K2, idx = big
    srv = B.Server(plan, precision="fp32", p_dtype="fp32", batch=1, n_sets=1, max_g=2, max_s=1, max_wait_ms=0.0)
    tk = [srv.submit(P, K1, K2, 2, 1, idx) for _ in range(4)]
    srv.cancel(tk[3])
    with pytest.raises(B.BlastError) as e:
        srv.wait(tk[3])
    assert e.value.status == B.E_CANCELLED
    polls, got = 0, None
    while got is None:
        got = srv.poll(tk[2])
        polls += 1
    for k in (0, 1):
        srv.wait(tk[k])
    with pytest.raises(B.BlastError) as e:
        srv.cancel(tk[0])
    assert e.value.status == B.E_INVALID
    st = srv.stats()
    srv.close()
    print("polls before completion", polls, flush=True)
    assert st["cancelled"] == 1 and st["completed"] == 3 and polls > 1
    ref = _direct(plan, (P, 2, 1, idx, K1, K2), "fp32", torch.float32)
    assert np.allclose(got[0], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


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
    # the binding checks the host tables it hands over: shape, dtype and the output array
    with pytest.raises(ValueError):
        srv.submit(P32, K1[:, :-1].copy(), K2, ng, ns, idx)
    with pytest.raises(ValueError):
        srv.submit(P32, K1, torch.as_tensor(K2).cuda(), ng, ns, idx)
    with pytest.raises(ValueError):
        srv.submit(P32, K1, K2, ng, ns, idx, out=np.empty((1, 1), dtype=np.float32))
    assert srv.stats()["submitted"] == 0
    srv.close()
