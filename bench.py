"""Throughput of the beyond-Limber 3x2pt C_ell path on one MI355X.

One step = the whole per-cosmology path (Chebyshev projection -> contraction with
the resident basis -> chi/R quadrature for every bin pair) over one batch of
synthetic cosmologies whose inputs are already resident in HBM.  The basis
precompute is done once before timing (as in the paper, where it is excluded from
the timings) and reported separately.

    python bench.py [--steps K] [--warmup W] [--batch B] [--precision fp32|fp16x3|bf16x3|fp64]

Prints ONE JSON line (see the keys at the bottom).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "3x2pt C_ell sets/sec at ≤1e-3 rel err vs FP64 oracle; p50/p99 latency"
PEAK = {"hbm": 8.0e12, "fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15, "fp16": 2.5e15}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16", "bf16": "bf16", "fp16x3": "f16x3"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def nodal_path(prec, cfg):
    """Whether the library contracts the nodal basis (the DCT applied to the basis when the plan
    is made) with nodal P itself, with no projection per call: FP16X3 on FP32 P with
    n_cheb % 4 == 0 and at most 16 bins; FP32 on FP32 P with n_cheb % 4 == 0; FP64 on FP64 P with
    n_cheb % 32 == 0 (the bench's P types)."""
    if prec == "fp16x3":
        return cfg.n_cheb % 4 == 0 and cfg.n_g + cfg.n_s <= 16
    if prec == "fp32":
        return cfg.n_cheb % 4 == 0
    return prec == "fp64" and cfg.n_cheb % 32 == 0


def stage_work(plan, cfg, prec, batch):
    """Algorithmic flops and HBM bytes of each stage for one launch over `batch` sets.

    projection : c = D P as the even/odd split DCT (two [N/2 x N/2] products per point): N^2
                 flops per (point, set); P read, c written once.  Absent on the nodal path,
                 whose contraction reads P in place of c.
    contraction: fused with the R-quadrature (w stays in registers; mixed paths, and the FP64
                 path at batches of 32 or more with at most 16 bins): basis and c read, weighted
                 kernels Kt written and read (from K_chi2; FP32 with the bins rounded up to a
                 multiple of 4, FP64 16 wide), Y written; flops of the contraction plus those of
                 the R-sum.  Unfused FP64: w = Ttilde c, basis read once per launch, c read, w
                 written.
    quad_R     : unfused FP64 only: w and K_chi2 read, Y written.
    quad_chi   : Y read, C written (negligible)."""
    NP = cfg.n_chi * cfg.n_R
    N = cfg.n_cheb
    rows = plan.rows
    rows_pad = plan.rows_pad
    nb = cfg.n_g + cfg.n_s
    nbp = 16 if nb <= 16 else 32
    eb = {"fp64": 8, "fp32": 4, "bf16": 2, "bf16x3": 4, "fp16x3": 4}[prec]  # basis bytes per element (hi+lo)
    ec = {"fp64": 8, "fp32": 4, "bf16": 2, "bf16x3": 4, "fp16x3": 4}[prec]  # coefficient bytes
    nodal = nodal_path(prec, cfg)
    es = 4 if prec == "fp16x3" and not nodal else 0  # coefficient row scale (projection -> Kt)
    ew = 8 if prec == "fp64" else 4                                    # w and Y bytes
    ep = 8 if prec == "fp64" else 4                                    # P bytes
    rows_bins = plan.n_ell * (cfg.n_g + nb + cfg.n_s)                 # (row, bin) products in the R-sum
    proj = dict(flops=(1.0 if N % 8 == 0 else 2.0) * NP * N * N * batch,
                bytes=float(NP * (N * (ep + ec) + es) * batch))
    quad_chi = dict(flops=4.0 * cfg.n_chi * plan.n_ell * B_pairs(cfg) * batch,
                    bytes=float(cfg.n_chi * rows_pad * nbp * ew * batch))
    y_bytes = float(cfg.n_chi * rows_pad * nbp * ew * batch)
    if prec == "fp64" and not fused_path(prec, nb, batch):
        out = {
            "projection": proj,
            "contraction": dict(flops=2.0 * rows * N * NP * batch,
                                bytes=float(NP * rows * N * eb + NP * N * ec * batch + NP * rows_pad * ew * batch)),
            "quad_R": dict(flops=2.0 * rows_bins * NP * batch,
                           bytes=float(NP * rows_pad * ew * batch + nb * NP * 8 * batch) + y_bytes),
            "quad_chi": quad_chi,
        }
        if nodal:
            del out["projection"]
        return out
    nbf = (nb + 3) // 4 * 4
    ek = 4  # weights table bytes per element
    if prec == "fp64":
        nbf, ek = 16, 8
    out = {
        "projection": proj,
        "r_weights": dict(flops=float(nb * NP * batch),
                          bytes=float(nb * NP * 8 * batch + NP * nbf * ek * batch + NP * es * batch)),
        "contraction": dict(flops=2.0 * rows * N * NP * batch + 2.0 * rows_bins * NP * batch,
                            bytes=float(NP * rows * N * eb + NP * N * ec * batch + NP * nbf * ek * batch) + y_bytes),
        "quad_chi": quad_chi,
    }
    if nodal:
        del out["projection"]
    return out


def fused_path(prec, nbins, batch):
    """Whether the library runs the contraction fused with the R-quadrature (no w_save): the
    mixed paths with at most 20 bins (FP16X3 at any batch, the others from batch 32), the FP64
    path with at most 16 bins from batch 32."""
    if prec == "fp64":
        return nbins <= 16 and batch >= 32
    return nbins <= 20 and (batch >= 32 or prec == "fp16x3")


def B_pairs(cfg):
    g, s = cfg.n_g, cfg.n_s
    return g * (g + 1) // 2 + g * s + s * (s + 1) // 2


def counter_traffic(kernel, cfg_name, batch, prec):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, when it
    was taken on the current kernel source, workload, batch and precision; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_2410_03632_amd", "csrc", "eval.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for r in rec.get("records", []):
        if (r["kernel"] == kernel and r["source_sha256"] == sha and r["workload"] == cfg_name
                and r["batch"] == batch and r["precision"] == prec):
            return r["fetch_bytes"] + r["write_bytes"]
    return None


def roofline(work, ms_per_launch, prec):
    flops, nbytes = work["flops"], work["bytes"]
    t = ms_per_launch * 1e-3
    peak_f = PEAK["fp64" if prec == "fp64" else ("bf16" if prec.startswith("bf16") else
                                                 ("fp16" if prec == "fp16x3" else "fp32"))]
    ridge = peak_f / PEAK["hbm"]
    if flops / nbytes >= ridge:
        a = flops / t / 1e12
        return {"bound": "mfma", "achieved": a, "peak": peak_f / 1e12, "unit": "TFLOP/s", "frac": a * 1e12 / peak_f,
                "traffic": None, "algorithmic_flops": flops, "algorithmic_bytes": nbytes}
    a = nbytes / t / 1e9
    return {"bound": "hbm", "achieved": a, "peak": PEAK["hbm"] / 1e9, "unit": "GB/s", "frac": a * 1e9 / PEAK["hbm"],
            "traffic": None, "algorithmic_flops": flops, "algorithmic_bytes": nbytes}


def cpu_model():
    """The host CPU's model name (first 'model name' line of /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_small_config(runs=3, st_chi=8):
    """The FP64 oracle on one whole set of the small named configuration (20 ell, 2 + 2 bins,
    chi 64 x R 32, 64 Chebyshev nodes) at its first k-panel level, `runs` times on all host
    cores (mean and standard deviation, the protocol of the paper's timing table), and once on
    one thread over `st_chi` of the 64 chi nodes (every R node of each), scaled by points."""
    import oracle as O
    from paper_2410_03632_amd import workloads as W
    cfg = W.CONFIGS[1]
    chi, wchi = O.grid_chi(cfg.n_chi, cfg.chi_min, cfg.chi_max)
    R, wR = O.grid_R(cfg.n_R, cfg.R_min)
    _, x = O.grid_k(cfg.n_cheb, cfg.k_min, cfg.k_max)
    k = np.exp(np.log(cfg.k_min) + 0.5 * (x + 1.0) * np.log(cfg.k_max / cfg.k_min))
    inp = W.make_inputs(cfg, W.seed_for(1, 0), k, chi, R)
    cores = O.max_threads()
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        O.cl_grid(cfg.ells(), ("gg", "gs", "ss"), cfg.k_min, cfg.k_max, cfg.n_cheb, chi, wchi, R, wR, inp.P,
                  cfg.n_g, cfg.n_s, inp.Kchi, inp.Kchi2, maxlev=1, nthreads=cores)
        ts.append(time.perf_counter() - t0)
    a = (np.arange(st_chi) * cfg.n_chi) // st_chi
    c1 = np.repeat(chi[a], cfg.n_R)
    c2 = (chi[a][:, None] * R[None, :]).ravel()
    t0 = time.perf_counter()
    O.w_points(cfg.ells(), ("gg", "gs", "ss"), cfg.k_min, cfg.k_max, c1, c2, nc=cfg.n_cheb,
               P=inp.P[a].reshape(-1, cfg.n_cheb), M=max(64, 2 * cfg.n_cheb), Phi=10.0, nthreads=1)
    t1 = (time.perf_counter() - t0) * cfg.n_chi / st_chi
    # the oracle keeps the last thread count it was given: back to all cores
    O.w_points(cfg.ells()[:1], ("gg",), cfg.k_min, cfg.k_max, c1[:1], c2[:1], nc=cfg.n_cheb,
               P=inp.P[a[0], 0], shared=True, nthreads=cores)
    return {"workload": "small named configuration: one whole set (20 ell, 10 pairs, chi 64 x R 32, 64 nodes), "
                        "the oracle's first k-panel level",
            "all_cores_s_per_set_mean": float(np.mean(ts)), "all_cores_s_per_set_std": float(np.std(ts)),
            "runs": runs, "cores": cores,
            "one_thread_s_per_set": t1,
            "one_thread_sample": "%d of 64 chi nodes (all 32 R nodes each), scaled by points" % st_chi}


def cpu_baseline(cfg, plan, inp, config, n_sample=144, seed=11):
    """The FP64 oracle on a stratified sample of (chi_a, R_b) points of the benchmark workload,
    with the same two k-panel levels its doubling test runs, scaled by points to one full set
    (an estimate: a whole set takes the oracle about two hours), next to a measured whole set of
    the small named configuration."""
    import oracle as O
    rng = np.random.default_rng(seed)
    a_idx = (np.arange(n_sample) * cfg.n_chi) // n_sample
    b_idx = rng.integers(0, cfg.n_R, n_sample)
    c1 = plan.chi[a_idx]
    c2 = plan.chi[a_idx] * plan.R[b_idx]
    P = inp.P[a_idx, b_idx]
    M0 = max(64, 2 * cfg.n_cheb)
    t0 = time.time()
    for M, Phi in ((M0, 10.0), (2 * M0, 5.0)):
        O.w_points(cfg.ells(), ("gg", "gs", "ss"), cfg.k_min, cfg.k_max, c1, c2, nc=cfg.n_cheb, P=P, M=M, Phi=Phi)
    t = time.time() - t0
    s_per_set = t * (cfg.n_chi * cfg.n_R) / n_sample
    out = {"value": 1.0 / s_per_set, "unit": "sets/s", "cores": O.max_threads(), "kind": "oracle",
           "sample": "%d of %d (chi_a, R_b) points (stratified in chi), k-integrals at the oracle's first two "
                     "refinement levels, %.1f s wall, scaled by points to one set (estimate)"
                     % (n_sample, cfg.n_chi * cfg.n_R, t),
           "s_per_set": s_per_set, "cpu": cpu_model()}
    gpath = os.path.join(ROOT, "tests", "golden", "c%d_oracle.json" % config)
    if os.path.exists(gpath):
        g = json.load(open(gpath))
        out["golden_whole_set"] = {"s": g.get("wall_s"), "threads": g.get("threads"),
                                   "what": "the oracle's whole set of this workload when the stored values were "
                                           "written (another host)"}
    out["small_config_measured"] = cpu_small_config()
    return out


def serving_run(seconds, rate_hz=200.0, batch=16, precision="fp32", pool=32):
    """The serving configuration: a Poisson stream of single-cosmology requests (3-15
    clustering and 1-5 shear bins, 20-200 of the 200 master multipoles each) through the
    continuous-batching server.  Host-side generation of a 12.6 MB P grid per request cannot
    keep up with 200 requests/s, so the requests' cosmologies cycle through a pool of
    `pool` seed-drawn ones."""
    import threading

    import torch
    from paper_2410_03632_amd import blast as B
    from paper_2410_03632_amd import workloads as W

    cfg = W.SERVING
    t0 = time.time()
    plan = B.plan_for_config(cfg, precisions=(precision,))
    build_s = time.time() - t0
    chi, chi2 = plan.eval_points()
    Kchi, Kchi2 = W.kernels(W.bins_of(cfg), chi, chi2)
    n = max(1, int(seconds * rate_hz))
    reqs = W.serving_requests(n, rate_hz)
    pdt = torch.float32 if precision != "fp64" else torch.float64
    Ps = []
    for i in range(min(pool, n)):
        t = torch.empty((cfg.n_chi, cfg.n_R, cfg.n_cheb), dtype=pdt, pin_memory=True)
        t.copy_(torch.as_tensor(W.p_grid(plan.k_nodes, chi, chi2, reqs[i].cosmo)))
        Ps.append(t)
    kcache = {}

    def kern(ng, ns):
        if (ng, ns) not in kcache:
            K1, K2 = W.request_kernels(Kchi, Kchi2, ng, ns, max_g=15)
            kcache[(ng, ns)] = (torch.as_tensor(K1).pin_memory(), torch.as_tensor(K2).pin_memory())
        return kcache[(ng, ns)]

    for r in reqs:
        kern(r.n_g, r.n_s)
    srv = B.Server(plan, precision=precision, p_dtype="fp64" if precision == "fp64" else "fp32", batch=batch,
                   n_sets=2, max_g=15, max_s=5, max_wait_ms=2.0)
    tickets = []
    waiter_done = []

    def waiter():
        k = 0
        while k < n:
            if k < len(tickets):
                srv.wait(tickets[k])
                k += 1
            else:
                time.sleep(0.0002)
        waiter_done.append(True)

    th = threading.Thread(target=waiter)
    th.start()
    t_start = time.perf_counter()
    t_next = t_start
    for i, r in enumerate(reqs):
        t_next += r.gap_s
        dt = t_next - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        K1, K2 = kern(r.n_g, r.n_s)
        tickets.append(srv.submit(Ps[i % len(Ps)], K1, K2, r.n_g, r.n_s, r.ell_idx))
        if (i + 1) % 2000 == 0:
            log("serving: %d of %d requests submitted" % (i + 1, n))
    th.join()
    st = srv.stats()
    srv.close()
    plan.close()
    return {"rate_hz": rate_hz, "requests": n, "seconds_of_arrivals": seconds, "p50_ms": st["p50_ms"],
            "p99_ms": st["p99_ms"],
            "throughput_req_s": st["completed"] / (st["span_ms"] * 1e-3) if st["span_ms"] else None,
            "mean_fill": st["mean_fill"], "launches": st["launches"], "batch_slots": batch,
            "max_sets_in_flight": st["max_sets_in_flight"], "set_bytes": st["set_bytes"],
            "completed": st["completed"], "rejected": st["rejected"],
            "precision": precision, "plan_build_s": build_s,
            "workload": "200 master ell on [2,1000], chi 256, R 96, 128 Chebyshev nodes; per request 3-15 "
                        "clustering + 1-5 shear bins and 20-200 ell, Poisson arrivals; cosmologies cycle "
                        "through %d seed-drawn ones" % len(Ps)}


def sweep_run(steps=5):
    """Grid sweeps after the paper's discussion section, on the full 3x2pt workload (FP32 path,
    batch 64): time per set against the number of Chebyshev nodes and the number of bins, and
    the accuracy (Delta chi^2 of Eq. dchi, with LSST-like noise) against clustering bin width
    with the default and a refined chi-R grid.  Benchmarks are the FP64 path (its parity with
    the oracle is pinned separately): for node counts, FP64 at 128 nodes; for bin widths,
    FP64 on the refined grid."""
    import dataclasses

    import torch
    from paper_2410_03632_amd import blast as B
    from paper_2410_03632_amd import metrics as M
    from paper_2410_03632_amd import workloads as W

    base = W.CONFIGS[2]
    Bn = 64
    dev = torch.device("cuda:0")
    cos0 = W.draw_cosmo(np.random.default_rng(W.seed_for(2, 0)))

    def run(cfg, plan, prec, bins, n_g, n_s, timed=True):
        chi, chi2 = plan.eval_points()
        Kchi, Kchi2 = W.kernels(bins, chi, chi2)
        pdt = torch.float64 if prec == "fp64" else torch.float32
        P = torch.as_tensor(W.p_grid(plan.k_nodes, chi, chi2, cos0), dtype=pdt, device=dev)[None]
        P = P.expand(Bn, -1, -1, -1).contiguous()
        K1 = torch.as_tensor(Kchi, device=dev)[None].expand(Bn, -1, -1).contiguous()
        K2 = torch.as_tensor(Kchi2, device=dev)[None].expand(Bn, -1, -1, -1).contiguous()
        C = plan.forward(P, K1, K2, n_g, n_s, precision=prec)
        ms = None
        if timed:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                plan.forward(P, K1, K2, n_g, n_s, precision=prec)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
        return C[0].cpu().numpy(), ms

    out = {"workload": "full 3x2pt shapes, FP32 path, batch 64 (times per set)"}
    # E5: Chebyshev nodes
    bins = W.bins_of(base)
    ref_plan = B.plan_for_config(base, precisions=("fp64", "fp32"))
    Cref, _ = run(base, ref_plan, "fp64", bins, base.n_g, base.n_s, timed=False)
    pairs = W.pair_list(base.n_g, base.n_s)
    ref_plan.close()
    rows = []
    for N in (96, 104, 112, 120, 128):
        cfg = dataclasses.replace(base, n_cheb=N)
        plan = B.plan_for_config(cfg, precisions=("fp32",))
        C, ms = run(cfg, plan, "fp32", bins, cfg.n_g, cfg.n_s)
        rows.append({"n_cheb": N, "us_per_set": 1e3 * ms / Bn,
                     "delta_chi2_vs_fp64_128_l200": M.delta_chi2(C, Cref, plan.ell, cfg.n_g, cfg.n_s, pairs,
                                                                 ell_max=200),
                     "delta_chi2_vs_fp64_128": M.delta_chi2(C, Cref, plan.ell, cfg.n_g, cfg.n_s, pairs)})
        log("sweep n_cheb", rows[-1])
        plan.close()
    out["chebyshev_nodes"] = rows
    # E6: number of bins (one plan; clustering bins 1..10 with 1 or 5 shear bins)
    plan = B.plan_for_config(base, precisions=("fp32",))
    rows = []
    for n_s in (1, 5):
        for n_g in (1, 2, 4, 6, 8, 10):
            bsel = W.bins_of(base)[:n_g] + W.bins_of(base)[base.n_g:base.n_g + n_s]
            _, ms = run(base, plan, "fp32", bsel, n_g, n_s)
            rows.append({"n_g": n_g, "n_s": n_s, "pairs": len(W.pair_list(n_g, n_s)), "us_per_set": 1e3 * ms / Bn})
            log("sweep bins", rows[-1])
    plan.close()
    out["bins"] = rows
    # E7: clustering bin width (sigma 150, 75, 37.5 Mpc), default grid and a refined grid
    fine = dataclasses.replace(base, n_chi=512, n_R=128)
    mid = dataclasses.replace(base, n_chi=384, n_R=112)
    pf = B.plan_for_config(fine, precisions=("fp64",))
    pm = B.plan_for_config(mid, precisions=("fp64",))
    pd = B.plan_for_config(base, precisions=("fp64", "fp32"))
    rows = []
    for f in (1.0, 0.5, 0.25):
        cfgw = dataclasses.replace(base, g_sigma=base.g_sigma * f)
        bw = W.bins_of(cfgw)
        Cb, _ = run(fine, pf, "fp64", bw, base.n_g, base.n_s, timed=False)
        Cm, _ = run(mid, pm, "fp64", bw, base.n_g, base.n_s, timed=False)
        C64, _ = run(base, pd, "fp64", bw, base.n_g, base.n_s, timed=False)
        C32, _ = run(base, pd, "fp32", bw, base.n_g, base.n_s, timed=False)
        d = lambda X, Y, lm=200: M.delta_chi2(X, Y, pd.ell, base.n_g, base.n_s, pairs, ell_max=lm)
        rows.append({"width": f, "benchmark": "FP64, chi 512 x R 128", "l_range": "l < 200 (all l)",
                     "delta_chi2_fp64_chi256_R96": (d(C64, Cb), d(C64, Cb, None)),
                     "delta_chi2_fp32_chi256_R96": (d(C32, Cb), d(C32, Cb, None)),
                     "delta_chi2_fp64_chi384_R112": (d(Cm, Cb), d(Cm, Cb, None)),
                     "delta_chi2_fp32_vs_fp64_same_grid": (d(C32, C64), d(C32, C64, None))})
        log("sweep width", rows[-1])
    pf.close()
    pm.close()
    pd.close()
    out["bin_width"] = rows
    return out


def adjoint_work(plan, cfg, batch):
    """Algorithmic flops and HBM bytes per launch of the kernels of the FP32 gradient step (a
    forward that keeps w and Y on the fused path, then the adjoint to dP, dK_chi and dK_chi2).

    contract_quad_kernel : the fused forward (as stage_work's contraction) plus the w it keeps
    adj_dy_mfma_kernel   : dY = S Ktil per row: dC, K_chi read; dY (FP32), S (FP64) written
    adj_kchi_kernel      : dK_chi = S^T Y: Y and S read, dK_chi written
    adj_w_mfma_kernel    : dw = Khat dY and dK_chi2 = dY^T w: w, dY, K_chi2 read; dw, dK_chi2 written
    contract_tiled_kernel: dc = Ttilde^T dw: transposed basis once, dw read, dc written; on the
                           nodal path (n_cheb % 32 == 0) dP = B^T dw with the transposed nodal
                           basis, written straight into dP
    adj_project_split_kernel: dP = D^T dc (even/odd split, N^2 flops per row): dc read, dP written
                           (not on the nodal path)"""
    NP = cfg.n_chi * cfg.n_R
    N, ncp, R, Rp = cfg.n_cheb, plan.nc_pad, plan.rows, plan.rows_pad
    nb = cfg.n_g + cfg.n_s
    NB = 16 if nb <= 16 else 32
    fwd = stage_work(plan, cfg, "fp32", batch)["contraction"]
    w_bytes = 4.0 * NP * Rp * batch
    dy_bytes = 4.0 * R * cfg.n_chi * NB * batch
    out = {
        "contract_quad_kernel": dict(flops=fwd["flops"], bytes=fwd["bytes"] + w_bytes),
        "adj_dy_mfma_kernel": dict(flops=2.0 * NB * NB * cfg.n_chi * R * batch,
                                   bytes=8.0 * batch * (B_pairs(cfg) * plan.n_ell + nb * cfg.n_chi) + dy_bytes
                                   + 8.0 * R * NB * NB * batch),
        "adj_kchi_kernel": dict(flops=2.0 * NB * NB * cfg.n_chi * R * batch,
                                bytes=dy_bytes + 8.0 * R * NB * NB * batch + 8.0 * nb * cfg.n_chi * batch),
        "adj_w_mfma_kernel": dict(flops=4.0 * NB * R * NP * batch,
                                  bytes=2 * w_bytes + dy_bytes + 16.0 * nb * NP * batch),
        "contract_tiled_kernel": dict(flops=2.0 * R * N * NP * batch,
                                      bytes=4.0 * NP * R * N + w_bytes + 4.0 * NP * ncp * batch),
        "adj_project_split_kernel": dict(flops=1.0 * N * N * NP * batch, bytes=4.0 * NP * (ncp + N) * batch),
    }
    if nodal_path("fp32", cfg):
        del out["adj_project_split_kernel"]
    return out


def gradient_run(plan, cfg, P, K1, K2, out, Bn, steps, warmup, dp_only=True):
    """The FP32 gradient step: a forward that keeps w, then the adjoint from dC = dL/dC to the
    gradients with respect to P at the nodes, K_chi and K_chi2, timed over `steps` calls."""
    import torch
    P32 = P if P.dtype == torch.float32 else P.float()
    wg = torch.empty(Bn * cfg.n_chi * cfg.n_R * plan.rows_pad, dtype=torch.float32, device=P.device)
    yg = torch.empty(plan.y_numel(Bn, cfg.n_g + cfg.n_s), dtype=torch.float32, device=P.device)
    outg = torch.empty_like(out)
    dC = torch.ones_like(out)

    def grad_step():
        plan.forward(P32, K1, K2, cfg.n_g, cfg.n_s, precision="fp32", out=outg, w_save=wg, y_save=yg)
        return plan.backward(P32, K1, K2, cfg.n_g, cfg.n_s, dC, precision="fp32", w_save=wg, y_save=yg)

    def grad_step_p():
        # dL/dP alone: the adjoint reads neither w nor Y, so the forward keeps nothing
        plan.forward(P32, K1, K2, cfg.n_g, cfg.n_s, precision="fp32", out=outg)
        return plan.backward(P32, K1, K2, cfg.n_g, cfg.n_s, dC, precision="fp32", want=("P",))

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps, r

    msg, grads = timed(grad_step)
    res = {"batch": Bn, "ms_per_step": msg, "sets_per_s": Bn / (msg * 1e-3),
           "kernel_work": adjoint_work(plan, cfg, Bn),
           "finite": bool(all(torch.isfinite(g).all().item() for g in grads if g is not None)),
           "what": "forward keeping w and Y + adjoint: dC -> dP (nodal), dK_chi, dK_chi2"}
    if dp_only:
        msp, gp = timed(grad_step_p)
        res["dP_only"] = {"ms_per_step": msp, "sets_per_s": Bn / (msp * 1e-3),
                          "finite": bool(torch.isfinite(gp[0]).all().item()),
                          "what": "forward keeping nothing + adjoint to dP alone"}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--precision", default="fp16x3", choices=["fp16x3", "fp32", "bf16x3", "fp64", "bf16"])
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP64-path and batch-1 timings")
    ap.add_argument("--serving-seconds", type=float, default=60.0, help="seconds of Poisson arrivals (0: skip)")
    ap.add_argument("--sweep", action="store_true", help="only run the grid sweeps (one JSON line)")
    ap.add_argument("--only-gradient", action="store_true",
                    help="only time the FP32 gradient step (forward keeping w, then the adjoint to dP, dK_chi and "
                         "dK_chi2) at --batch")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (asked for %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n}))
        return
    if args.sweep:
        print(json.dumps({"sweep": sweep_run()}), flush=True)
        return
    from paper_2410_03632_amd import blast as B
    from paper_2410_03632_amd import workloads as W
    from paper_2410_03632_amd.metrics import g16_err, error_by_pair

    cfg = W.CONFIGS[args.config]
    prec = args.precision
    log("building plan for config", args.config, cfg.name)
    t0 = time.time()
    precs = ("fp64", "fp32", "bf16x3", "bf16", "fp16x3")
    plan = B.plan_for_config(cfg, precisions=precs)
    build_s = time.time() - t0
    log("plan built in %.1f s (%d k-nodes, basis %s bytes)" % (build_s, plan.kq_nodes, plan.basis_bytes))

    # inputs: batch of seeded cosmologies, resident on the device
    Bn = args.batch
    chi, chi2 = plan.eval_points()
    Kchi, Kchi2 = W.kernels(W.bins_of(cfg), chi, chi2)
    inps = [W.make_inputs(cfg, W.seed_for(args.config, i), plan.k_nodes, plan.chi, plan.R) for i in range(min(Bn, 4))]
    rng_cos = [W.draw_cosmo(np.random.default_rng(W.seed_for(args.config, i))) for i in range(Bn)]
    dev = torch.device("cuda:0")
    pdt = torch.float64 if prec == "fp64" else torch.float32
    P = torch.empty((Bn, cfg.n_chi, cfg.n_R, cfg.n_cheb), dtype=pdt, device=dev)
    for i, cos in enumerate(rng_cos):
        P[i] = torch.as_tensor(W.p_grid(plan.k_nodes, chi, chi2, cos), dtype=pdt)
    K1 = torch.as_tensor(Kchi, device=dev).unsqueeze(0).expand(Bn, -1, -1).contiguous()
    K2 = torch.as_tensor(Kchi2, device=dev).unsqueeze(0).expand(Bn, -1, -1, -1).contiguous()
    out = torch.empty((Bn, B.n_pairs(cfg.n_g, cfg.n_s), plan.n_ell), dtype=torch.float64, device=dev)
    ws = torch.empty(plan.workspace_bytes(Bn, prec, cfg.n_g + cfg.n_s), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def step():
        plan.forward(P, K1, K2, cfg.n_g, cfg.n_s, precision=prec, out=out, workspace=ws)

    if args.only_gradient:
        print(json.dumps({"gradient_fp32": gradient_run(plan, cfg, P, K1, K2, out, Bn, args.steps, args.warmup,
                                                        dp_only=False)}), flush=True)
        plan.close()
        return

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.profile(True)
    plan.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.profile(False)
    stage_ms, ncalls = plan.profile_read()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = Bn / (ms_per_step * 1e-3)
    per_launch = {k: v / max(ncalls, 1) for k, v in stage_ms.items()}
    fused = fused_path(prec, cfg.n_g + cfg.n_s, Bn)
    if fused:
        # intervals of the fused path: R-quadrature weights, then contraction + R-quadrature
        per_launch = {"projection": per_launch["projection"], "r_weights": per_launch["contraction"],
                      "contraction": per_launch["quad_R"], "quad_chi": per_launch["quad_chi"]}
    if nodal_path(prec, cfg):
        del per_launch["projection"]  # nothing runs there
    log("ms/step %.3f  sets/s %.1f  stages(ms/launch) %s" % (ms_per_step, value, per_launch))
    work = stage_work(plan, cfg, prec, Bn)
    dom = max(per_launch, key=per_launch.get)
    roof = roofline(work[dom], per_launch[dom], prec)
    split = {"fp64": "project_split64_kernel", "fp16x3": "project_h16_kernel"}.get(prec, "project_split_kernel")
    kernel_of = {"projection": split if cfg.n_cheb % 8 == 0 else "project_kernel",
                 "contraction": (("contract_quad_f64_kernel" if prec == "fp64" else
                                  "contract_quad_wide_kernel" if prec == "fp16x3" and cfg.n_g + cfg.n_s <= 16
                                  else "contract_quad_kernel") if fused else "contract_kernel"),
                 "quad_R": "quad_y_kernel", "quad_chi": "quad_c_mfma_kernel", "r_weights": "kt_kernel"}
    roof["kernel"] = kernel_of[dom]
    roof["traffic"] = counter_traffic(roof["kernel"], cfg.name, Bn, prec)
    roof["stage_ms_per_launch"] = per_launch
    roof["stage_roofline"] = {k: roofline(work[k], per_launch[k], prec) for k in per_launch if k in work}
    for k, v in roof["stage_roofline"].items():
        v.pop("algorithmic_flops", None)
        v.pop("algorithmic_bytes", None)
        v["kernel"] = kernel_of[k]
        v["traffic"] = counter_traffic(kernel_of[k], cfg.name, Bn, prec)
    # the whole step against HBM: every stage's algorithmic bytes (including the R-weights table
    # and Y, which one stage writes and the next reads) over the step's wall time
    step_bytes = float(sum(work[k]["bytes"] for k in per_launch if k in work))
    roof["step"] = {"algorithmic_bytes": step_bytes, "achieved": step_bytes / (ms_per_step * 1e-3) / 1e9,
                    "peak": 8000.0, "unit": "GB/s", "frac": step_bytes / (ms_per_step * 1e-3) / 8e12}

    # accuracy of the timed path: cosmology 0 (the stored oracle values' cosmology) against them
    res = out[0].cpu().numpy()
    err = {}
    gold = None
    gpath = os.path.join(ROOT, "tests", "golden", "c%d_oracle.json" % args.config)
    if os.path.exists(gpath):
        g = json.load(open(gpath))
        if g["seed"] == W.seed_for(args.config, 0):
            gold = np.array(g["C"])
            err["max_rel_err_vs_oracle"] = float(g16_err(res, gold, cfg.n_g, cfg.n_s).max())
    # per bin pair error of every precision against the oracle (the largest per pair type and the
    # worst pairs), each from a call over the timed batch whose cosmology 0 is the stored one
    perr = {}
    if gold is not None:
        perr[prec] = error_by_pair(res, gold, cfg.n_g, cfg.n_s, plan.ell)
    extras = {}
    if not args.no_extras:
        # FP64 path on the same batch (the mixed-vs-FP64 speedup compares equal work), and
        # single-cosmology latency of the timed path
        P64 = torch.as_tensor(inps[0].P[None], device=dev)
        r64 = plan.forward(P64, K1[:1].contiguous(), K2[:1].contiguous(), cfg.n_g, cfg.n_s, precision="fp64")
        torch.cuda.synchronize()
        if "max_rel_err_vs_oracle" not in err:
            e = g16_err(res, r64[0].cpu().numpy(), cfg.n_g, cfg.n_s)
            err["max_rel_err_vs_fp64_path"] = float(e.max())
        nb64 = Bn
        P64b = P[:nb64].double().contiguous()
        P64b[0] = P64[0]  # cosmology 0 with its FP64 P, the oracle's input
        out64 = torch.empty((nb64,) + tuple(out.shape[1:]), dtype=torch.float64, device=dev)
        for _ in range(2):
            plan.forward(P64b, K1[:nb64].contiguous(), K2[:nb64].contiguous(), cfg.n_g, cfg.n_s, precision="fp64",
                         out=out64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            plan.forward(P64b, K1[:nb64].contiguous(), K2[:nb64].contiguous(), cfg.n_g, cfg.n_s, precision="fp64",
                         out=out64)
        torch.cuda.synchronize()
        ms64 = (time.perf_counter() - t0) * 1e3 / 5
        extras["fp64_path"] = {"batch": nb64, "ms_per_step": ms64, "sets_per_s": nb64 / (ms64 * 1e-3),
                               "kernel": "contract_quad_f64_kernel" if fused_path("fp64", cfg.n_g + cfg.n_s, nb64)
                               else "contract_kernel"}
        if gold is not None:
            r0 = out64[0].cpu().numpy()
            extras["fp64_path"]["max_rel_err_vs_oracle"] = float(g16_err(r0, gold, cfg.n_g, cfg.n_s).max())
            perr["fp64"] = error_by_pair(r0, gold, cfg.n_g, cfg.n_s, plan.ell)
        del out64, P64b
        extras["mixed_vs_fp64_speedup"] = value / extras["fp64_path"]["sets_per_s"]
        if prec != "fp32":
            # the FP32 path on the same batch: throughput, its fused kernel's roofline, its error
            P32 = P if P.dtype == torch.float32 else P.float()
            for _ in range(2):
                plan.forward(P32, K1, K2, cfg.n_g, cfg.n_s, precision="fp32", out=out)
            torch.cuda.synchronize()
            plan.profile(True)
            plan.profile_read()
            t0 = time.perf_counter()
            for _ in range(5):
                plan.forward(P32, K1, K2, cfg.n_g, cfg.n_s, precision="fp32", out=out)
            torch.cuda.synchronize()
            ms32 = (time.perf_counter() - t0) * 1e3 / 5
            plan.profile(False)
            st32, n32 = plan.profile_read()
            pl32 = {k: v / max(n32, 1) for k, v in st32.items()}
            pl32 = {"projection": pl32["projection"], "r_weights": pl32["contraction"],
                    "contraction": pl32["quad_R"], "quad_chi": pl32["quad_chi"]}
            if nodal_path("fp32", cfg):
                del pl32["projection"]
            r32 = roofline(stage_work(plan, cfg, "fp32", Bn)["contraction"], pl32["contraction"], "fp32")
            r32.pop("algorithmic_bytes", None)
            r32["traffic"] = counter_traffic("contract_quad_kernel", cfg.name, Bn, "fp32")
            f32 = {"batch": Bn, "ms_per_step": ms32, "sets_per_s": Bn / (ms32 * 1e-3), "stage_ms_per_launch": pl32,
                   "fused_kernel_roofline": r32}
            if gold is not None:
                r0 = out[0].cpu().numpy()
                f32["max_rel_err_vs_oracle"] = float(g16_err(r0, gold, cfg.n_g, cfg.n_s).max())
                perr["fp32"] = error_by_pair(r0, gold, cfg.n_g, cfg.n_s, plan.ell)
            extras["fp32_path"] = f32
        if gold is not None:
            P32 = P if P.dtype == torch.float32 else P.float()
            for pr in ("fp16x3", "bf16x3", "bf16"):
                if pr not in perr:
                    plan.forward(P32, K1, K2, cfg.n_g, cfg.n_s, precision=pr, out=out)
                    perr[pr] = error_by_pair(out[0].cpu().numpy(), gold, cfg.n_g, cfg.n_s, plan.ell)
        step()  # out holds the timed path's result again
        torch.cuda.synchronize()
        # differentiation at the same batch (FP32): a forward that keeps w, then the adjoint from
        # dC = dL/dC to the gradients with respect to P at the nodes, K_chi and K_chi2
        extras["gradient_fp32"] = gradient_run(plan, cfg, P, K1, K2, out, Bn, 5, 2)
        P1, K11, K21 = P[:1].contiguous(), K1[:1].contiguous(), K2[:1].contiguous()
        lat = []
        for i in range(12):
            torch.cuda.synchronize()
            ta = time.perf_counter()
            plan.forward(P1, K11, K21, cfg.n_g, cfg.n_s, precision=prec)
            torch.cuda.synchronize()
            if i >= 2:
                lat.append((time.perf_counter() - ta) * 1e3)
        extras["batch1_latency_ms"] = {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))}
        # sets/s of the timed path over batch sizes (inputs tiled from the timed batch)
        sweep = {}
        for nbat in (1, 8, 64, 256):
            reps = (nbat + Bn - 1) // Bn
            Pb = P.repeat(reps, 1, 1, 1)[:nbat].contiguous()
            K1b = K1[:1].expand(nbat, -1, -1).contiguous()
            K2b = K2[:1].expand(nbat, -1, -1, -1).contiguous()
            for _ in range(2):
                plan.forward(Pb, K1b, K2b, cfg.n_g, cfg.n_s, precision=prec)
            torch.cuda.synchronize()
            nrep = 3 if nbat >= 64 else 10
            t0 = time.perf_counter()
            for _ in range(nrep):
                plan.forward(Pb, K1b, K2b, cfg.n_g, cfg.n_s, precision=prec)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / nrep
            sweep[str(nbat)] = {"ms_per_step": ms, "sets_per_s": nbat / (ms * 1e-3)}
            del Pb, K1b, K2b
        extras["batch_sweep"] = sweep
        # Limber correction of the same batch: extended Limber of P_nl - P_lin at the Limber points
        kl = plan.limber_k()
        PL = torch.empty((Bn, plan.n_ell, cfg.n_chi), dtype=torch.float64, device=dev)
        PN = torch.empty_like(PL)
        for i, cos in enumerate(rng_cos):
            PL[i] = torch.as_tensor(W.p_limber(kl, chi, cos))
            PN[i] = torch.as_tensor(W.p_limber(kl, chi, cos, nonlinear=True))
        for _ in range(2):
            plan.limber(PN, K1, cfg.n_g, cfg.n_s, P_sub=PL, order=2, out=out, accumulate=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            plan.limber(PN, K1, cfg.n_g, cfg.n_s, P_sub=PL, order=2, out=out, accumulate=True)
        torch.cuda.synchronize()
        extras["limber_correction_ms_per_step"] = (time.perf_counter() - t0) * 1e3 / 5
        # one GPU's share of an 8-way split over multipoles (basis rows are independent, so G GPUs
        # would each hold 1/G of the rows): every 8th multipole, same grids, same batch
        ells = cfg.ells()[::8]
        tb = time.time()
        ps = B.Plan(ells, plan.chi, plan.w_chi, plan.R, plan.w_R, cfg.k_min, cfg.k_max, cfg.n_cheb, precisions=(prec,))
        tb = time.time() - tb
        for _ in range(2):
            ps.forward(P, K1, K2, cfg.n_g, cfg.n_s, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            ps.forward(P, K1, K2, cfg.n_g, cfg.n_s, precision=prec)
        torch.cuda.synchronize()
        ms_s = (time.perf_counter() - t0) * 1e3 / 10
        extras["multipole_slice_of_8"] = {"n_ell": len(ells), "batch": Bn, "ms_per_step": ms_s,
                                          "sets_per_s_of_the_slice": Bn / (ms_s * 1e-3), "plan_build_s": tb}
        ps.close()

    serving = None
    if args.serving_seconds > 0:
        log("serving run: %.1f s of arrivals at 200 requests/s" % args.serving_seconds)
        plan.close()
        # the server runs the FP32 path: at its small batches the unfused kernels are faster
        serving = serving_run(args.serving_seconds, precision="fp32")
        log("serving: %s" % serving)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        cpu = cpu_baseline(cfg, plan, inps[0], args.config)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "sets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[prec],
        "data": "synthetic",
        "config": {"workload": "full 3x2pt: %d clustering + %d shear bins (%d pairs), %d ell in [%d, %d], "
                               "chi %d on [%g, %g] Mpc, R %d on [%g, 1], %d Chebyshev nodes in ln k on [%g, %g]"
                               % (cfg.n_g, cfg.n_s, B.n_pairs(cfg.n_g, cfg.n_s), cfg.n_ell, cfg.ell_min,
                                  cfg.ell_max, cfg.n_chi, cfg.chi_min, cfg.chi_max, cfg.n_R, cfg.R_min,
                                  cfg.n_cheb, cfg.k_min, cfg.k_max),
                   "batch": Bn, "precision": prec, "basis_build_s": build_s, "kq_nodes": plan.kq_nodes},
        "roofline": roof,
        "cpu_baseline": cpu,
        # the paper's own timing, as context only: another grid (N5K fiducial), another machine
        "paper_context": {"ms_per_set": 3.60, "sets_per_s": 278, "precision": "f64",
                          "hardware": "2x AMD EPYC 7532, 32 threads (CPU)", "grid": "N5K fiducial, not config 2"},
    }
    line.update(err)
    if perr:
        line["error_by_precision"] = {
            "what": "cosmology 0 of the timed batch against the oracle's stored values: element-wise relative "
                    "error (cross spectra floored at 1e-3 of the geometric mean of the two auto spectra), the "
                    "largest per pair type and the three worst pairs with the multipole of their peak",
            "batch": Bn, **perr}
    line.update(extras)
    if serving:
        line["p50_ms"] = serving["p50_ms"]
        line["p99_ms"] = serving["p99_ms"]
        line["serving"] = serving
    print(json.dumps(line), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
