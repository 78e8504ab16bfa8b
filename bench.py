#!/usr/bin/env python3
"""Benchmark of the filter-diagonalization (FD) hot path on one MI355X.

A step is one FD outer iteration on the 3D Anderson lattice L=200 (D = 8.0M,
7-point hopping t=1, periodic, disorder W=16.5 drawn with seed 1), target
"nearest E = 0", with N_s search vectors in bundles of nb = 64 (default
N_s = 64, one bundle; --ns 512 for the full search space):
  coefficients (Jackson-damped delta at E=0, degree 500, host)
  -> Chebyshev filter (500 fused SpMMV steps per bundle)
  -> SVQB2 orthogonalization (MFMA Gram + GPU Jacobi + MFMA rotation)
  -> Rayleigh-Ritz (one more SpMMV per bundle, Gram, Jacobi, rotations,
     residual norms) -> selection of the pairs nearest E = 0 (host).
Inputs (matrix and the N(0,1) start block) are resident in HBM before the
timed region.  `value` is the whole step's algorithmic bytes (Eq. traffic,
with kappa = 5 for the steps that update V and kappa = 3 for the others --
V takes two terms every other step -- plus the dense passes) divided by the
step's wall time.

Extra fields: a SpMMV / filter bandwidth sweep over nb and precision, for
the CSR matrix and the same matrix in SELL-32-1, with the device STREAM
ceilings (copy, triad, read-only, write-only); the FD
eigenpairs/s comparison FP64 vs mixed precision on the Hubbard ring L=8 and
L=14 (the mixed-precision workload: 64 pairs in [-1, 1], per-pair errors of
the mixed run against the FP64 run); the roofline of the dominant kernel
(the fused Chebyshev step) and the CPU oracle baseline (host STREAM, SpMMV
per nb, filter and FD samples).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SpMMV GB/s (% of HBM peak); FD eigenpairs/s at residual 1e-9, mixed vs FP64"
HBM_PEAK_GBS = 8000.0


T_START = time.time()


def log(*a):
    print("[bench] %6.1fs" % (time.time() - T_START), *a, file=sys.stderr, flush=True)


# ----------------------------------------------------------- byte counts ----
def spmmv_bytes(nnz, D, nb, sv):
    """Eq. traffic at N_p = 1: matrix (value + uint32 index), row pointers,
    X read once, Y written once."""
    return nnz * (sv + 4) + 4 * (D + 1) + 2 * D * nb * sv


def fused_bytes(nnz, D, nb, sv, kappa=5):
    """Fused Chebyshev step: W1 read once, W2 and V read and written."""
    return nnz * (sv + 4) + 4 * (D + 1) + kappa * D * nb * sv


def filter_step_counts(degree):
    """Steps 3..n of the filter: (steps with the V update, kappa = 5; steps
    with the recurrence only, kappa = 3).  V is updated with two terms at
    every even step, and at an odd last step."""
    n_even = degree // 2 - 1
    n_last = 1 if degree % 2 == 1 and degree >= 3 else 0
    return n_even + n_last, (degree - 2) - n_even - n_last


def filter_bytes(nnz, D, nb, sv, degree):
    """One filter application on one bundle: step 1 (SpMMV + write), step 2
    (kappa = 4: gather, read V, write W1 and V), then the steps with the V
    update (kappa = 5: W1 read once, W2 and V read and written) and the
    recurrence-only steps (kappa = 3)."""
    n5, n3 = filter_step_counts(degree)
    return (fused_bytes(nnz, D, nb, sv, 2) + fused_bytes(nnz, D, nb, sv, 4)
            + n5 * fused_bytes(nnz, D, nb, sv, 5) + n3 * fused_bytes(nnz, D, nb, sv, 3))


def dense_bytes(D, ns):
    """SVQB2 (2 Gram reads + 2 in-place rotations) and Rayleigh-Ritz (Gram of
    V and W, two rotations, residual norms), FP64."""
    blk = D * ns * 8
    return 2 * blk + 2 * 2 * blk + 2 * blk + 2 * 2 * blk + 2 * blk


# ------------------------------------------------------------- helpers ----
def traffic_from_profile(kernel_src: str, site_order: str):
    """HBM bytes per launch of the fused step from the committed rocprofv3
    PMC summary, if it was taken on the current kernel source and the same
    site numbering of the matrix."""
    path = os.path.join(ROOT, "profiles", "chebyshev_steps_anderson200_nb64_f64_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        prof = json.load(f)
    h = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    if prof.get("kernel_source_sha256") != h or prof.get("site_order") != site_order:
        return None
    return prof.get("hbm_bytes_per_launch"), prof.get("launch_shape")


def fd_runs(args, fd, np):
    """FD to residual 1e-9 ||H||, FP64 filter vs FP32 filter (mixed), same
    start block, window, degree and interval rule; eigenpairs per second.
    Per pair: |lambda_mixed - lambda_FP64| / ||H|| and both residuals."""
    from fd_inputs import start_block
    fdres = {}
    # (name, model, window, N_t, N_s, nb, degree)
    runs = [("hubbard8", dict(L=8, n_up=4, n_dn=4, U=4.0), -0.5, 0.5, 16, 128, 16, 100)]
    if not args.no_hub14:
        runs.append(("hubbard14", dict(L=14, n_up=7, n_dn=7, U=8.0), -1.0, 1.0, 64, 256, 32, 800))
    # one line per FD iteration on stderr (the L=14 solves run for minutes)
    os.environ["FD_TRACE"] = "1"
    for name, kw, lo, hi, nt, nsr, nbr, deg in runs:
        t0 = time.time()
        mh = fd.build_matrix("hubbard", fmt=args.hub_fmt, t=1.0, config_order=args.hub_order, **kw)
        log("FD %s: matrix built in %.1fs (D=%d)" % (name, time.time() - t0, mh.D))
        V0 = start_block(mh.D, nsr, 0) if mh.D * nsr <= 50_000_000 else None
        res = {}
        out = {}
        for prec, label in ((0, "fp64"), (1, "mixed")):
            r = fd.solve(mh, lo, hi, nt, nsr, nbr, deg, max_iter=40, tol=1e-9, precision=prec, V0=V0,
                         seed=0, want_vectors=False, adapt=args.adapt)
            st = r.stats
            res[label] = {"converged": r.status == fd.FD_OK, "eigenpairs_per_s": round(nt / st["t_total"], 4),
                          "t_total_s": round(st["t_total"], 3), "iters": st["iters"],
                          "iters_fp32": st["iters_fp32"], "spmmv": st["spmmv_count"],
                          "t_filter_s": round(st["t_filter"], 3), "t_orthog_s": round(st["t_orthog"], 3),
                          "t_rr_s": round(st["t_rr"], 3), "max_resid_rel": st["max_resid"] / st["norm_H"],
                          "norm_H": st["norm_H"]}
            out[label] = r
            log("FD %s %s: %s" % (name, label, res[label]))
        normH = res["fp64"]["norm_H"]
        e64, emx = out["fp64"].evals, out["mixed"].evals
        res["config"] = {"D": mh.D, "nnz": mh.nnz, "format": args.hub_fmt, "labels": ["ranked", "rcm"][args.hub_order],
                         "window": [lo, hi], "n_target": nt, "n_search": nsr, "nb": nbr, "degree": deg,
                         "window_rule": {0: "fixed", 1: "ritz", 2: "lehmann"}[args.adapt]}
        res["per_pair"] = {"eval_fp64": [float(x) for x in e64],
                           "abs_diff_mixed_vs_fp64_rel": [float(abs(a - b) / normH) for a, b in zip(emx, e64)],
                           "resid_fp64_rel": [float(x / normH) for x in out["fp64"].resid],
                           "resid_mixed_rel": [float(x / normH) for x in out["mixed"].resid]}
        res["mixed_vs_fp64_max_rel_eval_diff"] = max(res["per_pair"]["abs_diff_mixed_vs_fp64_rel"])
        res["E0_found"] = bool(np.abs(e64).min() <= 1e-10 * normH and np.abs(emx).min() <= 1e-10 * normH)
        res["speedup_mixed_over_fp64"] = round(res["fp64"]["t_total_s"] / res["mixed"]["t_total_s"], 3)
        log("FD %s: mixed/FP64 speedup %.3f, max |dlambda|/||H|| %.2e, E=0 found %s"
            % (name, res["speedup_mixed_over_fp64"], res["mixed_vs_fp64_max_rel_eval_diff"], res["E0_found"]))
        if mh.D <= 100_000:
            # the same solves with CholQR2 orthogonalization (SVQB2 where a
            # Cholesky pass fails); eigenvalues against the SVQB2 FP64 run
            res["cholqr2"] = {}
            for prec, label in ((0, "fp64"), (1, "mixed")):
                r = fd.solve(mh, lo, hi, nt, nsr, nbr, deg, max_iter=40, tol=1e-9, precision=prec, V0=V0,
                             seed=0, want_vectors=False, adapt=args.adapt, ortho=fd.FD_ORTHO_CHOLQR2)
                st = r.stats
                res["cholqr2"][label] = {
                    "converged": r.status == fd.FD_OK, "eigenpairs_per_s": round(nt / st["t_total"], 4),
                    "t_total_s": round(st["t_total"], 3), "iters": st["iters"], "spmmv": st["spmmv_count"],
                    "t_filter_s": round(st["t_filter"], 3), "t_orthog_s": round(st["t_orthog"], 3),
                    "t_rr_s": round(st["t_rr"], 3), "max_resid_rel": st["max_resid"] / st["norm_H"],
                    "max_rel_eval_diff_vs_svqb2_fp64": float(np.abs(r.evals - e64).max() / normH)
                    if r.evals.size == e64.size else None}
                log("FD %s %s CholQR2: %s" % (name, label, res["cholqr2"][label]))
        fdres[name] = res
        del mh
    return fdres


def batch_runs(args, fd, np, torch):
    """Batched workload: 96 3D Anderson instances drawn from SplitMix64 seeds
    100-195 (L in [20, 64], W in [2, 20)), 16 pairs nearest E = 0 each,
    N_s = 64.  (1) One degree-200 filter application (damped delta at E = 0)
    on every instance: batched (one graph replay) against one instance after
    another, algorithmic GB/s.  (2) FD to 1e-9 ||H|| on instances drawn the
    same way at L in [8, 16] (the full-size instances need filter degrees of
    10^4 and more near E = 0): batched against one fd_solve per instance,
    eigenpairs/s and p50/p99 time per instance."""
    from fd_inputs import anderson_batch
    out = {}
    ns, degree = 64, 200
    # one line per batched FD iteration on stderr (the full-size solve runs for minutes)
    os.environ["FD_TRACE"] = "1"
    inst = anderson_batch(range(100, 196))
    t0 = time.time()
    mats = [fd.build_matrix(**q) for q in inst]
    b = fd.Batch(mats)
    log("batch: 96 instances, D_total=%d, built in %.1fs" % (b.D, time.time() - t0))
    alpha = [2.0 / (m.lam_hi - m.lam_lo) for m in mats]
    beta = [-(m.lam_hi + m.lam_lo) / (m.lam_hi - m.lam_lo) for m in mats]
    mu = [fd.cheb_coeffs(1, bt, 0.0, degree) for bt in beta]
    degs = [degree] * len(mats)
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    V = torch.randn((b.D, ns), generator=g, dtype=torch.float64, device="cuda")
    W1 = torch.empty_like(V)
    W2 = torch.empty_like(V)

    def alg_bytes(nb):
        return sum(degree * (ns // nb) * (m.nnz * 12 + 4 * (m.D + 1) + 5 * m.D * nb * 8) for m in mats)

    # nb and the launch shape chosen by the library (fd_batch_autotune)
    t = time.perf_counter()
    nb, chunk, sh = fd.batch_autotune(b, "f64", 0)
    t_tune = time.perf_counter() - t
    log("batch autotune: nb %d, XCD chunk %d rows, entry loop %d (%.1fs)" % (nb, chunk, sh, t_tune))
    times = {}
    fd.batch_filter(b, V, mu, degs, alpha, beta, W1, W2, nb)  # graph capture
    torch.cuda.synchronize()
    reps = 3
    t = time.perf_counter()
    for _ in range(reps):
        fd.batch_filter(b, V, mu, degs, alpha, beta, W1, W2, nb)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t) / reps
    # one instance after another, same nb, fd_cheb_filter per instance
    t = time.perf_counter()
    for i, m in enumerate(mats):
        r = slice(int(b.off[i]), int(b.off[i + 1]))
        fd.cheb_filter(m, V[r], mu[i], alpha[i], beta[i], W1[r], W2[r], nb)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t
    out["filter_full"] = {"instances": len(mats), "D_total": b.D, "n_search": ns, "degree": degree, "nb": nb,
                          "autotuned": {"nb": nb, "chunk_rows": chunk, "entry_loop": sh, "tune_s": round(t_tune, 2)},
                          "batched_s": round(tb, 4), "sequential_s": round(ts, 4),
                          "batched_GBs": round(alg_bytes(nb) / tb / 1e9, 1),
                          "sequential_GBs": round(alg_bytes(nb) / ts / 1e9, 1),
                          "speedup": round(ts / tb, 2)}
    log("batch filter: %s" % out["filter_full"])
    del V, W1, W2
    torch.cuda.empty_cache()

    # (1b) FD at the full sizes, as specified: 16 pairs nearest E = 0 per
    # instance, the KPM rule's degree (capped), N_s = 64, nb chosen by the
    # library, a few outer iterations; converged count and eigenpairs/s
    nt = 16
    t = time.perf_counter()
    degs_full = [min(args.batch_max_degree, fd.pick_degree(m, 0.0, 0.0, nt, ns)[0]) for m in mats]
    log("FD full size: KPM-rule degrees in [%d, %d] (cap %d), %.1fs"
        % (min(degs_full), max(degs_full), args.batch_max_degree, time.perf_counter() - t))
    params = [dict(tau_lo=0.0, tau_hi=0.0, n_target=nt, n_search=ns, nb=0, degree=d, max_iter=args.batch_full_iters,
                   tol=1e-9, seed=2000 + i) for i, d in enumerate(degs_full)]
    r = fd.solve_batch(b, params)
    conv = [s_["iters"] <= args.batch_full_iters and s_["max_resid"] <= 1e-9 * s_["norm_H"] for s_ in r.stats]
    tconv = sorted(s_["t_total"] for s_, c in zip(r.stats, conv) if c)
    out["fd_full"] = {"instances": len(mats), "D_total": b.D, "n_target": nt, "n_search": ns,
                      "nb": r.bstats["nb"], "degree_range": [min(degs_full), max(degs_full)],
                      "max_iter": args.batch_full_iters, "converged": int(sum(conv)),
                      "t_total_s": round(r.bstats["t_total"], 2),
                      "eigenpairs_per_s": round(nt * sum(conv) / r.bstats["t_total"], 3),
                      "p50_completion_s": round(float(np.percentile(tconv, 50)), 2) if tconv else None,
                      "p99_completion_s": round(float(np.percentile(tconv, 99)), 2) if tconv else None,
                      "max_resid_rel_median": float(np.median([s_["max_resid"] / s_["norm_H"] for s_ in r.stats]))}
    log("FD full size: %s" % out["fd_full"])
    del b, mats
    torch.cuda.empty_cache()

    # (2) FD on small instances drawn the same way, with both orthogonalizations
    inst = anderson_batch(range(100, 196), L_lo=8, L_span=9)
    mats = [fd.build_matrix(**q) for q in inst]
    nt, ns, nb = 16, 64, 16
    degs = [fd.pick_degree(m, 0.0, 0.0, nt, ns)[0] for m in mats]
    log("FD batch: degrees from the KPM rule in [%d, %d]" % (min(degs), max(degs)))
    b = fd.Batch(mats)
    out["fd_small"] = {"instances": len(mats), "D_total": b.D, "L": [min(q["L"] for q in inst),
                                                                       max(q["L"] for q in inst)],
                       "n_target": nt, "n_search": ns, "nb": nb, "degree_range": [min(degs), max(degs)]}
    for oname, ortho in (("svqb2", fd.FD_ORTHO_SVQB2), ("cholqr2", fd.FD_ORTHO_CHOLQR2)):
        params = [dict(tau_lo=0.0, tau_hi=0.0, n_target=nt, n_search=ns, nb=nb, degree=d,
                       max_iter=args.batch_iters, tol=1e-9, seed=1000 + i, ortho=ortho) for i, d in enumerate(degs)]
        r = fd.solve_batch(b, params)
        conv = [s["iters"] <= args.batch_iters and s["max_resid"] <= 1e-9 * s["norm_H"] for s in r.stats]
        tconv = sorted(s["t_total"] for s, c in zip(r.stats, conv) if c)
        res = {"batched": {"converged": int(sum(conv)), "t_total_s": round(r.bstats["t_total"], 3),
                           "eigenpairs_per_s": round(nt * sum(conv) / r.bstats["t_total"], 2),
                           "p50_completion_s": round(float(np.percentile(tconv, 50)), 3) if tconv else None,
                           "p99_completion_s": round(float(np.percentile(tconv, 99)), 3) if tconv else None,
                           "iters": r.bstats["iters"], "t_filter_s": round(r.bstats["t_filter"], 3),
                           "t_orthog_s": round(r.bstats["t_orthog"], 3), "t_rr_s": round(r.bstats["t_rr"], 3),
                           "graph_launches": r.bstats["graph_launches"]}}
        log("batched FD (%s): %s" % (oname, res["batched"]))
        ev_b = r.evals
        tl, done_at, nconv, maxdiff = [], [], 0, 0.0
        t = time.perf_counter()
        for i, m in enumerate(mats):
            q = params[i]
            s1 = fd.solve(m, 0.0, 0.0, nt, ns, nb, q["degree"], max_iter=q["max_iter"], tol=1e-9, seed=q["seed"],
                          ortho=ortho, want_vectors=False)
            if i % 32 == 31:
                log("sequential FD (%s): %d of %d instances done" % (oname, i + 1, len(mats)))
            if s1.status == fd.FD_OK:
                nconv += 1
                tl.append(s1.stats["t_total"])
                done_at.append(time.perf_counter() - t)
                if conv[i]:
                    maxdiff = max(maxdiff, float(np.max(np.abs(s1.evals - ev_b[i])) / s1.stats["norm_H"]))
        tseq = time.perf_counter() - t
        res["sequential"] = {"converged": nconv, "t_total_s": round(tseq, 3),
                             "eigenpairs_per_s": round(nt * nconv / tseq, 2),
                             "p50_completion_s": round(float(np.percentile(done_at, 50)), 3) if done_at else None,
                             "p99_completion_s": round(float(np.percentile(done_at, 99)), 3) if done_at else None,
                             "p50_solve_s": round(float(np.percentile(tl, 50)), 3) if tl else None,
                             "p99_solve_s": round(float(np.percentile(tl, 99)), 3) if tl else None}
        res["speedup_batched_over_sequential"] = round(tseq / r.bstats["t_total"], 2)
        res["max_rel_eval_diff_batched_vs_single"] = maxdiff
        log("sequential FD (%s): %s" % (oname, res["sequential"]))
        out["fd_small"][oname] = res
    return out


def hubbard16_runs(args, fd, np, torch):
    """Matrix-free SpMMV and Chebyshev steps on the Hubbard ring L=16, 8 up +
    8 down (D = 165,636,900, the dimension of the paper's Hubbard16), U = 25,
    8 FP64 vectors: the setting of the paper's matrix-free per-SpMV timing on
    one CPU node (Sec. 4.2)."""
    t0 = time.time()
    m = fd.build_matrix("hubbard", fmt="matfree", L=16, n_up=8, n_dn=8, t=1.0, U=25.0)
    log("Hubbard L=16 matrix-free: D=%d nnz=%d (not stored), tables in %.1fs" % (m.D, m.nnz, time.time() - t0))
    out = {"D": m.D, "nnz": m.nnz, "format": "matfree", "U": 25.0}
    for dt, name, nb in ((torch.float64, "f64", 8), (torch.float64, "f64", 32), (torch.float32, "f32", 8)):
        shape = fd.autotune(m, name, nb)
        X = torch.randn((m.D, nb), dtype=dt, device="cuda")
        Y = torch.empty_like(X)
        fd.spmmv(m, X, Y)
        torch.cuda.synchronize()
        reps = 10
        t = time.perf_counter()
        for _ in range(reps):
            fd.spmmv(m, X, Y)
        torch.cuda.synchronize()
        t_spmmv = (time.perf_counter() - t) / reps
        alpha, beta = 2.0 / (m.lam_hi - m.lam_lo), -(m.lam_hi + m.lam_lo) / (m.lam_hi - m.lam_lo)
        W1, W2 = torch.empty_like(X), torch.empty_like(X)
        deg = 20
        mu = fd.cheb_coeffs(1, beta, 0.0, deg)
        t = time.perf_counter()
        fd.cheb_filter(m, X, mu, alpha, beta, W1, W2, nb)
        torch.cuda.synchronize()
        t_step = (time.perf_counter() - t) / deg
        key = "%s_nb%d" % (name, nb)
        out[key] = {"spmmv_ms": round(t_spmmv * 1e3, 2), "filter_step_ms": round(t_step * 1e3, 2),
                    "launch_shape": list(shape)}
        log("Hubbard L=16 %s: %s" % (key, out[key]))
        del X, Y, W1, W2
        torch.cuda.empty_cache()
    out["paper_context"] = "2.04 s per SpMV with 8 FP64 vectors on one CPU node, matrix-free (Sec. 4.2)"
    return out


def cpu_baseline(args, np, L, nb, alpha, beta, fdres):
    """The oracle on the host cores beside the GPU run (Sec. 3.2's STREAM b_m
    and kappa, measured on the host): a bounded sample of about 20-30 s.
    Headline value: the unfused FP64 filter on one nb-wide bundle of the
    Anderson workload (degree --cpu-degree), in the same algorithmic GB/s as
    the GPU's.  Extras: host STREAM triad, SpMMV per nb, one full filter of
    the Hubbard L=8 workload, its FD solve, and the per-step time of the
    Hubbard L=14 filter with the FD time extrapolated from it."""
    import platform
    import subprocess
    # threads pinned one per core, the -O3 x86-64-v3 copy of the oracle
    os.environ.setdefault("OMP_PLACES", "cores")
    os.environ.setdefault("OMP_PROC_BIND", "close")
    os.environ["FD_ORACLE_FAST"] = "1"
    import oracle as O
    from fd_inputs import start_block
    res = {}
    try:
        lscpu = subprocess.run(["lscpu", "-p=CORE,SOCKET"], capture_output=True, text=True).stdout
        cores = {tuple(x.split(",")) for x in lscpu.splitlines() if x and not x.startswith("#")}
        res["host_physical_cores"] = len(cores)
    except OSError:
        res["host_physical_cores"] = None
    res["host_cpu"] = platform.processor() or platform.machine()

    def med(f, n=3):
        f()
        ts = []
        for _ in range(n):
            t0 = time.perf_counter()
            f()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    # host STREAM triad on 3 x 1 GiB
    n = 1 << 27
    a, b, c = np.ones(n), np.full(n, 2.0), np.empty(n)
    t = med(lambda: O.stream_triad(a, b, c, 0.5))
    bm = 3 * n * 8 / t / 1e9
    res["stream_triad_GBs"] = round(bm, 2)
    del a, b, c
    t0 = time.time()
    A = O.anderson(L, 1.0, 16.5, 1)
    log("cpu: oracle Anderson matrix built in %.1fs, STREAM triad %.1f GB/s" % (time.time() - t0, bm))
    D, nnz = A.D, A.rowptr[-1]
    # SpMMV per nb (natural numbering)
    sp = {}
    for w in (1, 4, 8, 16, 32, 64):
        X = np.random.default_rng(0).standard_normal((D, w))
        ts = med(lambda: O.spmmv(A, X), 2)
        sp[str(w)] = {"s": round(ts, 4), "GBs": round(spmmv_bytes(nnz, D, w, 8) / ts / 1e9, 2)}
        del X
    res["spmmv_anderson"] = sp
    log("cpu: SpMMV %s" % sp)
    # headline: the unfused filter on one bundle
    Vc = np.random.default_rng(0).standard_normal((D, nb))
    mu = O.cheb_coeffs(1, beta, 0.0, args.cpu_degree)
    t0 = time.perf_counter()
    O.cheb_filter(A, Vc, mu, alpha, beta)
    tc = time.perf_counter() - t0
    cb = filter_bytes(nnz, D, nb, 8, args.cpu_degree)
    # the paper's kappa from the same run: vector traffic per step and row
    # and vector at the STREAM bandwidth, after the matrix bytes
    step_t = tc / args.cpu_degree
    res["kappa_host"] = round((step_t * bm * 1e9 - (nnz * 12 + 4 * (D + 1))) / (D * nb * 8), 2)
    res.update({"value": round(cb / tc / 1e9, 2), "unit": "GB/s", "cores": O.num_threads(), "kind": "oracle",
                "sample": "unfused FP64 filter, degree %d, one bundle of nb=%d on Anderson L=%d (natural site "
                          "numbering; %.1f s); same algorithmic byte count as the GPU filter"
                          % (args.cpu_degree, nb, L, tc)})
    del Vc, A
    # the remaining samples only while the whole run stays well inside its
    # time limit
    if time.time() - T_START > args.cpu_deadline:
        res["skipped"] = "Hubbard samples (run time past %d s)" % args.cpu_deadline
        return res
    # Hubbard L=8: one full filter (degree 100, N_s = 128) and the FD solve
    H8 = O.hubbard(8, 4, 4, 1.0, 4.0)
    a8, b8 = O.scaling(*O.gershgorin(H8))
    V8 = start_block(H8.D, 128, 0)
    res["filter_hubbard8_s"] = round(med(lambda: O.cheb_filter(H8, V8, O.cheb_coeffs(0, a8 * -0.5 + b8,
                                                                                     a8 * 0.5 + b8, 100),
                                                              a8, b8), 2), 4)
    t0 = time.perf_counter()
    r8 = O.fd_solve(H8, V8, -0.5, 0.5, 16, 100, 1e-9, max_iter=80, adapt=1)
    res["fd_hubbard8"] = {"s": round(time.perf_counter() - t0, 3), "iters": r8.iters, "converged": r8.converged,
                          "eigenpairs_per_s": round(16 / (time.perf_counter() - t0), 3)}
    log("cpu: Hubbard L=8 filter %.3fs, FD %s" % (res["filter_hubbard8_s"], res["fd_hubbard8"]))
    # Hubbard L=14: two steps of the filter on one bundle of 32, extrapolated
    if not args.no_hub14 and time.time() - T_START < args.cpu_deadline:
        t0 = time.time()
        H14 = O.hubbard(14, 7, 7, 1.0, 8.0)
        a14, b14 = O.scaling(*O.gershgorin(H14))
        X = np.random.default_rng(0).standard_normal((H14.D, 32))
        t0 = time.perf_counter()
        O.cheb_filter(H14, X, O.cheb_coeffs(0, b14 - a14, b14 + a14, 2), a14, b14)
        t2 = (time.perf_counter() - t0) / 2
        g = fdres.get("hubbard14", {}).get("fp64", {})
        n_spmmv = g.get("spmmv")
        res["hubbard14"] = {"step_s_nb32": round(t2, 3),
                            "filter_s_extrapolated": round(t2 * 800 * 8, 1),
                            "fd_s_extrapolated": round(t2 * n_spmmv, 1) if n_spmmv else None,
                            "note": "per-step time of the oracle's unfused filter on one bundle of 32 (2 steps "
                                    "timed); filter = 800 steps x 8 bundles; FD = the GPU FP64 run's SpMMV count "
                                    "x step time (T_FD ~ n_SpMV T_SpMV, Sec. 4.3), extrapolated"}
        log("cpu: Hubbard L=14 %s" % res["hubbard14"])
        del H14, X
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--L", type=int, default=200)
    ap.add_argument("--nb", type=int, default=64)
    ap.add_argument("--ns", type=int, default=64)
    ap.add_argument("--degree", type=int, default=500)
    ap.add_argument("--fmt", choices=["csr", "sell", "pencil"], default="csr",
                    help="storage / walk of the Anderson matrix (pencil: (x, y) tiles of C x sigma over all z)")
    ap.add_argument("--tiles", default="100x40",
                    help="Anderson site numbering: TXxTY numbers sites along (x, y) tiles over all z, 0 = natural")
    ap.add_argument("--C", type=int, default=32)
    ap.add_argument("--sigma", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-sweep", action="store_true", help="skip the nb / precision sweep")
    ap.add_argument("--no-fd", action="store_true", help="skip the FD eigenpairs/s runs")
    ap.add_argument("--no-hub14", action="store_true",
                    help="skip the FD runs on the Hubbard ring L=14 (the mixed-precision workload)")
    ap.add_argument("--hub-order", type=int, choices=[0, 1], default=1,
                    help="Hubbard basis labels of the FD runs: 0 ranked, 1 reverse Cuthill-McKee (the same "
                         "operator, P A P^T)")
    ap.add_argument("--site-compare", action="store_true",
                    help="also time a degree-20 filter with the tiled and the natural Anderson numbering")
    ap.add_argument("--fd-only", action="store_true", help="only the FD eigenpairs/s runs (no Anderson step)")
    ap.add_argument("--hubbard16", action="store_true",
                    help="only the matrix-free SpMMV / filter step on the Hubbard ring L=16 (D = 165.6M)")
    ap.add_argument("--batch", action="store_true",
                    help="only the batched workload (96 Anderson instances; filter and FD, batched vs one by one)")
    ap.add_argument("--batch-iters", type=int, default=80, help="max outer iterations per batched FD instance")
    ap.add_argument("--batch-full-iters", type=int, default=3,
                    help="outer iterations of the batched FD at the full instance sizes")
    ap.add_argument("--batch-max-degree", type=int, default=12000,
                    help="cap on the KPM-rule degree of the batched FD at the full instance sizes")
    ap.add_argument("--adapt", type=int, choices=[0, 1, 2], default=1,
                    help="filter window of the FD runs: 0 fixed, 1 tracked by the N_t-th Ritz value, "
                         "2 tracked by the Lehmann radius")
    ap.add_argument("--hub-fmt", choices=["csr", "sell", "matfree"], default="csr",
                    help="storage of the Hubbard matrices in the FD runs (matfree: tensor-product form, "
                         "fastest at nb <= 8; csr at nb >= 32)")
    ap.add_argument("--cpu-degree", type=int, default=6, help="filter degree of the CPU sample")
    ap.add_argument("--cpu-deadline", type=int, default=440,
                    help="skip the CPU baseline's Hubbard samples once the run has taken this many seconds")
    ap.add_argument("--pmc-sample-hubbard14", action="store_true",
                    help="short run for hardware counters on the mixed-precision workload's step: one 1 GiB "
                         "STREAM copy, then one degree-12 filter on one nb=32 bundle of the Hubbard ring L=14, "
                         "FP64 and FP32, in the --hub-fmt storage and --hub-order labels; prints the sizes")
    ap.add_argument("--pmc-sample", action="store_true",
                    help="short run for hardware counters: one 1 GiB STREAM copy, then one degree-12 "
                         "filter and five plain SpMMVs on one nb=64 FP64 bundle of the workload; prints the sizes "
                         "and exits")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path; "
              "the filter's sharding across GPUs is a design, not code.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2209_01974_amd as fd

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    if args.pmc_sample_hubbard14:
        n = 1 << 27  # 1 GiB of doubles
        a = torch.ones(n, dtype=torch.float64, device=dev)
        c = torch.empty_like(a)
        fd.stream(0, a, c, stream=stream)
        torch.cuda.synchronize()
        del a, c
        mh = fd.build_matrix("hubbard", fmt=args.hub_fmt, L=14, n_up=7, n_dn=7, t=1.0, U=8.0,
                             config_order=args.hub_order)
        al, be = 2.0 / (mh.lam_hi - mh.lam_lo), -(mh.lam_hi + mh.lam_lo) / (mh.lam_hi - mh.lam_lo)
        res = {"pmc_sample_hubbard14": True, "copy_bytes_read": n * 8, "copy_bytes_written": n * 8,
               "D": mh.D, "nnz": mh.nnz, "nb": 32, "format": args.hub_fmt,
               "labels": ["ranked", "rcm"][args.hub_order], "launches_mode5": 5, "launches_mode4": 5}
        for dt, name, sv in ((torch.float64, "f64", 8), (torch.float32, "f32", 4)):
            res["shape_" + name] = list(fd.autotune(mh, name, 32, stream=stream))
            V1 = torch.randn((mh.D, 32), dtype=dt, device=dev)
            Z1, Z2 = torch.empty_like(V1), torch.empty_like(V1)
            fd.cheb_filter(mh, V1, fd.cheb_coeffs(1, be, 0.0, 12), al, be, Z1, Z2, 32, stream=stream)
            torch.cuda.synchronize()
            res["algorithmic_bytes_mode5_" + name] = fused_bytes(mh.nnz, mh.D, 32, sv, 5)
            res["algorithmic_bytes_mode4_" + name] = fused_bytes(mh.nnz, mh.D, 32, sv, 3)
            del V1, Z1, Z2
        print(json.dumps(res), flush=True)
        return
    if args.fd_only:
        print(json.dumps({"fd": fd_runs(args, fd, np)}), flush=True)
        return
    if args.batch:
        print(json.dumps({"batch": batch_runs(args, fd, np, torch)}), flush=True)
        return
    if args.hubbard16:
        print(json.dumps({"hubbard16": hubbard16_runs(args, fd, np, torch)}), flush=True)
        return

    # ---------------------------------------------------------- workload ----
    L, nb, ns, degree = args.L, args.nb, args.ns, args.degree
    t0 = time.time()
    tiles = (0, 0) if args.tiles in ("0", "") or args.fmt == "pencil" else tuple(int(v) for v in args.tiles.split("x"))
    m = fd.build_matrix("anderson", fmt=args.fmt, C_=args.C, sigma=args.sigma, L=L, t=1.0, W=16.5, seed=1,
                        tiles=tiles)
    D, nnz = m.D, m.nnz
    site_order = "(x, y) tiles %dx%d over all z" % tiles if tiles[0] else "natural (x + L y + L^2 z)"
    log("built Anderson L=%d D=%d nnz=%d (%s, sites %s) in %.1fs" % (L, D, nnz, args.fmt, site_order,
                                                                     time.time() - t0))
    lam_lo, lam_hi = m.lam_lo, m.lam_hi
    alpha, beta = 2.0 / (lam_hi - lam_lo), -(lam_hi + lam_lo) / (lam_hi - lam_lo)
    g = torch.Generator(device=dev)
    g.manual_seed(0)
    if args.pmc_sample:
        n = 1 << 27  # 1 GiB of doubles
        a = torch.ones(n, dtype=torch.float64, device=dev)
        c = torch.empty_like(a)
        fd.stream(0, a, c, stream=stream)
        torch.cuda.synchronize()
        shape = fd.autotune(m, "f64", nb, stream=stream)
        V1 = torch.randn((D, nb), generator=g, dtype=torch.float64, device=dev)
        Z1, Z2 = torch.empty_like(V1), torch.empty_like(V1)
        fd.cheb_filter(m, V1, fd.cheb_coeffs(1, beta, 0.0, 12), alpha, beta, Z1, Z2, nb, stream=stream)
        for _ in range(5):  # plain SpMMV (MODE 0), same launch shape
            fd.spmmv(m, V1, Z1, stream=stream)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_sample": True, "launch_shape": list(shape), "copy_bytes_read": n * 8,
                          "copy_bytes_written": n * 8,
                          "launches_mode5": 5, "launches_mode4": 5, "launches_mode0": 5,
                          "algorithmic_bytes_mode5": fused_bytes(nnz, D, nb, 8, 5),
                          "algorithmic_bytes_mode4": fused_bytes(nnz, D, nb, 8, 3),
                          "algorithmic_bytes_mode0": spmmv_bytes(nnz, D, nb, 8),
                          "D": D, "nnz": nnz, "nb": nb}), flush=True)
        return
    shape = fd.autotune(m, "f64", nb, stream=stream)
    log("autotuned launch shape (order, xcd, iters, grid, nontemporal): %s" % (shape,))
    V = torch.randn((D, ns), generator=g, dtype=torch.float64, device=dev)
    W = torch.empty_like(V)
    W1 = torch.empty((D, nb), dtype=torch.float64, device=dev)
    W2 = torch.empty_like(W1)
    nbund = ns // nb
    torch.cuda.synchronize()

    def step(record=None):
        mu = fd.cheb_coeffs(1, alpha * 0.0 + beta, 0.0, degree)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fd.cheb_filter(m, V, mu, alpha, beta, W1, W2, nb, stream=stream)
        e1.record(stream)
        fd.orthog(V, fd.FD_ORTHO_SVQB2, seed=7, stream=stream)
        th, rho = fd.rayleigh_ritz(m, V, W, nb, stream=stream)
        order = np.argsort(np.abs(th), kind="stable")[:min(128, ns)]
        torch.cuda.synchronize()
        if record is not None:
            record.append(e0.elapsed_time(e1) * 1e-3)
        return th[order], rho[order]

    fd.orthog(V, fd.FD_ORTHO_SVQB2, seed=7, stream=stream)
    torch.cuda.synchronize()
    for i in range(args.warmup):
        step()
        log("warmup step %d done" % i)
    filt_times = []
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for i in range(args.steps):
        th, rho = step(filt_times)
        log("step %d: filter %.3fs, min |theta| %.3e, max rho(%d nearest 0) %.3e"
            % (i, filt_times[-1], np.abs(th).min(), len(th), rho.max()))
    torch.cuda.synchronize()
    te = time.perf_counter()
    t_step = (te - ts) / args.steps
    fb = filter_bytes(nnz, D, nb, 8, degree) * nbund
    step_bytes = fb + nbund * spmmv_bytes(nnz, D, nb, 8) + dense_bytes(D, ns)
    value = step_bytes / t_step / 1e9

    # roofline of the dominant kernel: the Chebyshev step kernel (HIP events
    # around each filter call on the launch stream; every launch in it is the
    # SpMMV/Chebyshev kernel: per bundle the two first steps, then the steps
    # alternate between the recurrence only (MODE 4) and the recurrence with
    # the two-term V update (MODE 5)); bytes and time are per average launch
    t_filter = sum(filt_times) / len(filt_times)
    launches = degree * nbund
    avg_launch = t_filter / launches
    achieved = fb / t_filter / 1e9
    per_launch = fb / launches
    traffic, traffic_shape = None, None
    if (L, nb, args.fmt) == (200, 64, "csr"):
        tp = traffic_from_profile(os.path.join(ROOT, "paper_2209_01974_amd", "csrc", "fd_spmmv.hip"), site_order)
        if tp is not None:
            traffic, traffic_shape = tp
    n5, n3 = filter_step_counts(degree)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_spmmv<double,2,32,MODE 4|5> (Chebyshev steps, FP64, nb=64; per launch averaged "
                          "over a filter application: %d steps with the V update, %d without, 2 first steps)"
                          % (n5, n3),
                "algorithmic_bytes_per_launch": round(per_launch), "avg_launch_us": round(avg_launch * 1e6, 2),
                "traffic_launch_shape": traffic_shape}
    del W
    torch.cuda.empty_cache()

    out = {"metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(t_step * 1e3, 1), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "anderson3d_L%d_W16.5_seed1" % L, "D": D, "nnz": nnz,
                      "n_search": ns, "nb": nb, "degree": degree, "format": args.fmt, "site_order": site_order,
                      "target": "%d pairs nearest E=0 (damped delta)" % min(128, ns), "parallelism": "single GPU",
                      "launch_shape": list(shape)},
           "roofline": roofline,
           "hbm_frac_of_step": round(value / HBM_PEAK_GBS, 4)}

    # ------------------------------------------- site numbering check ----
    # the same degree-20 filter on one bundle with the tiled and the natural
    # numbering of the lattice (each with its autotuned launch shape)
    if tiles[0] and args.site_compare:
        mn = fd.build_matrix("anderson", L=L, t=1.0, W=16.5, seed=1)
        cmp_ = {}
        for name, mm in (("tiled", m), ("natural", mn)):
            sh = fd.autotune(mm, "f64", nb, stream=stream)
            X = torch.empty((D, nb), dtype=torch.float64, device=dev).normal_(generator=g)
            Z1, Z2 = torch.empty_like(X), torch.empty_like(X)
            mu = fd.cheb_coeffs(1, beta, 0.0, 20)
            fd.cheb_filter(mm, X, mu, alpha, beta, Z1, Z2, nb, stream=stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fd.cheb_filter(mm, X, mu, alpha, beta, Z1, Z2, nb, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            tf = e0.elapsed_time(e1) * 1e-3
            cmp_[name] = {"step_us": round(tf / 20 * 1e6, 1), "GBs": round(filter_bytes(nnz, D, nb, 8, 20) / tf / 1e9, 1),
                          "launch_shape": list(sh)}
            del X, Z1, Z2
        del mn
        out["site_order_compare"] = cmp_
        log("degree-20 filter, nb=%d: tiled %.0f us, natural %.0f us per step"
            % (nb, cmp_["tiled"]["step_us"], cmp_["natural"]["step_us"]))

    # ---------------------------------------------------------- sweep ----
    if not args.no_sweep:
        sweep = []
        # device STREAM (the paper's b_m measurement): copy and triad on 4 GB arrays
        a = torch.empty(D * 64, dtype=torch.float64, device=dev).normal_()
        b = torch.empty_like(a).normal_()
        c = torch.empty_like(a)
        for op, name, nbytes in ((0, "stream_copy_GBs", 2), (1, "stream_triad_GBs", 3), (2, "stream_read_GBs", 1),
                                 (3, "stream_write_GBs", 1)):
            for _ in range(3):
                fd.stream(op, a, c, b, 0.5, stream=stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(10):
                fd.stream(op, a, c, b, 0.5, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            out[name] = round(nbytes * a.numel() * 8 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
        log("STREAM copy %.0f GB/s, triad %.0f GB/s, read-only %.0f GB/s, write-only %.0f GB/s"
            % (out["stream_copy_GBs"], out["stream_triad_GBs"], out["stream_read_GBs"], out["stream_write_GBs"]))
        del a, b, c
        # the benchmark's matrix (CSR, tiled numbering), and the same matrix in
        # SELL-32-1 (chunks of 32 rows, no sorting: the rows of a chunk read
        # entry j from consecutive addresses), which serves small nb better
        m_sell = fd.build_matrix("anderson", fmt="sell", C_=32, sigma=1, L=L, t=1.0, W=16.5, seed=1, tiles=tiles)
        for fmt_name, mm in (("csr", m), ("sell-32-1", m_sell)):
            for dt, sv in ((torch.float64, 8), (torch.float32, 4)):
                for w in (1, 4, 8, 16, 32, 64):
                    shape_w = fd.autotune(mm, "f64" if sv == 8 else "f32", w, stream=stream)
                    X = torch.empty((D, w), dtype=dt, device=dev).normal_()
                    Y = torch.empty_like(X)
                    for _ in range(3):
                        fd.spmmv(mm, X, Y, stream=stream)
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    reps = 20
                    e0.record(stream)
                    for _ in range(reps):
                        fd.spmmv(mm, X, Y, stream=stream)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    ts_ = e0.elapsed_time(e1) * 1e-3 / reps
                    # algorithmic bytes count the nnz entries (padding slots of
                    # SELL are overhead; the lattice at L=200 has none)
                    gbs = spmmv_bytes(nnz, D, w, sv) / ts_ / 1e9
                    # filter of degree 50 on one bundle of width w
                    Z1, Z2 = torch.empty_like(X), torch.empty_like(X)
                    mu = fd.cheb_coeffs(1, beta, 0.0, 50)
                    fd.cheb_filter(mm, X, mu, alpha, beta, Z1, Z2, w, stream=stream)
                    e0.record(stream)
                    fd.cheb_filter(mm, X, mu, alpha, beta, Z1, Z2, w, stream=stream)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    tf = e0.elapsed_time(e1) * 1e-3
                    fgbs = filter_bytes(nnz, D, w, sv, 50) / tf / 1e9
                    sweep.append({"format": fmt_name, "dtype": "f64" if sv == 8 else "f32", "nb": w,
                                  "spmmv_us": round(ts_ * 1e6, 1), "spmmv_GBs": round(gbs, 1),
                                  "spmmv_frac": round(gbs / HBM_PEAK_GBS, 4),
                                  "filter_step_us": round(tf / 50 * 1e6, 1), "filter_GBs": round(fgbs, 1),
                                  "filter_frac": round(fgbs / HBM_PEAK_GBS, 4), "launch_shape": list(shape_w),
                                  "stored_entries": mm.stored})
                    log("sweep %s %s nb=%d: SpMMV %.0f GB/s, filter %.0f GB/s"
                        % (fmt_name, sweep[-1]["dtype"], w, gbs, fgbs))
                    del X, Y, Z1, Z2
        del m_sell
        torch.cuda.empty_cache()
        out["sweep"] = sweep

    # ---------------------------------------------------- FD eigenpairs/s ----
    if not args.no_fd:
        out["fd"] = fd_runs(args, fd, np)

    # ------------------------------------------------------- CPU oracle ----
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args, np, L, nb, alpha, beta, out.get("fd", {}))

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
