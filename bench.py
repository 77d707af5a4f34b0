#!/usr/bin/env python
"""Benchmark of the VIF hot path on one MI355X.

Step = one evaluation of the Gaussian VIF negative log-likelihood and its
gradient w.r.t. (variance, range, nugget) at n = 100,000 (d = 2, Matern-3/2
variance 1 range 0.05, nugget 0.05, m = 200 inducing points, m_v = 20
correlation neighbours): Sigma_m Cholesky, whitening, per-point factor,
Woodbury/Sylvester reduction, adjoint gradient. Inputs are resident in HBM
before the timed region; the neighbour search runs once before it (as in the
paper, neighbour selection is not part of a likelihood evaluation).

Prints one JSON line. ``value`` is FP32-form evaluations per second; the
FP64 form is reported beside it under "fp64".

Second leg ("laplace"): Laplace mode finding for a Bernoulli-logit latent VIF
model at n = 200,000 in [0,1]^5 (ARD Gaussian kernel, length scales
0.2..0.6, m = 500 kMeans++ inducing points, m_v = 30), Newton with
VIFDU-preconditioned CG to relative residual 1e-6, from the zero start and
from the learned warm start (feature and network time included). The network
is trained before the timed region on modes the method computes for three
other problems of the same shape.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "VIF NLL+grad evals/sec at n=100k (FP32 vs FP64); Laplace mode time, PCG iters"
HBM_PEAK_GBS = 8000.0


def factor_bytes_per_point(m: int, mv: int, d: int, tsize: int) -> int:
    """Algorithmic HBM bytes of the per-point factor kernel for one point with
    m_v neighbours: gather (m_v + 1) rows of V, the neighbour indices and the
    m_v + 1 coordinates; write the U row, A_i, D_i and the m_v(m_v+1)/2
    entries of the rows of L_R kept for the adjoint."""
    return (mv + 1) * m * tsize + mv * 4 + (mv + 1) * d * 8 + m * tsize + mv * tsize + 8 + mv * (mv + 1) // 2 * tsize


def factor_bwd_bytes_per_point(m: int, mv: int, d: int, tsize: int) -> int:
    """Algorithmic HBM bytes of the adjoint factor kernel for one point: gather
    the (m_v + 1) rows of V and of V_rho (the range derivative of V), read the
    point's U and Ubar rows, the neighbour indices, the m_v + 1 coordinates,
    the m_v responses of the neighbours, e_i, yt_i, D_i, A_i and the stored
    rows of L_R; write the three coefficient rows (S + G, sqrt(D) G,
    sqrt(D) beta) and three gradient partials."""
    return (2 * (mv + 1) * m * tsize + 2 * m * tsize + mv * 4 + (mv + 1) * d * 8 + mv * 8 + 24
            + mv * tsize + mv * (mv + 1) // 2 * tsize + 3 * m * tsize + 24)


def pcg_iter_bytes(n: int, m: int, mv: int) -> int:
    """Algorithmic HBM bytes of one VIFDU-preconditioned CG iteration (FP64):
    the operator (W + Sigma_dagger^{-1}) p passes over U twice (U^T t, U c) and
    over the sparse factor twice (B w, B^T s); the preconditioner passes over U
    twice (U^T q, U c) and over the factor twice (B^{-T}, B^{-1}); a pass over
    the factor reads m_v coefficients (8 B) and indices (4 B) per row; 41
    n-vector reads and writes of the recurrences and diagonal scalings."""
    return 4 * n * m * 8 + 4 * n * mv * 12 + 41 * n * 8


def measured_traffic(kernel: str = "k_factor"):
    """HBM bytes per launch of `kernel` (k_factor or k_factor_bwd, FP32, C2)
    from the committed counter summary, if it was taken on the current kernel
    source (else None)."""
    import hashlib
    try:
        txt = open(os.path.join(ROOT, "profiles", f"{kernel}_fp32_c2_pmc.md")).read()
        src = open(os.path.join(ROOT, "paper_2507_05064_amd", "csrc", "factor.hip"), "rb").read()
    except OSError:
        return None
    vals = {}
    for line in txt.splitlines():
        line = line.strip().lstrip("- ")
        for key in ("traffic_bytes_per_launch", "source_sha256"):
            if line.startswith(key):
                vals[key] = line.split(":", 1)[1].strip().split()[-1]
    if vals.get("source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return float(vals["traffic_bytes_per_launch"]) if "traffic_bytes_per_launch" in vals else None


def run_form(w, Xd, Zd, nbr, yd, precision, steps, warmup, grad):
    import torch
    from paper_2507_05064_amd.vif import VifContext
    ctx = VifContext(w.n, w.d, w.m, w.m_v, kernel=w.kernel, likelihood=w.likelihood, precision=precision,
                     tau_m=w.tau_m)
    theta = w.theta
    nth = theta.size

    def step():
        ctx.build_factor(Xd, Zd, nbr, theta)
        if grad:
            return ctx.nll_grad(yd, nth)
        return ctx.nll(yd), None

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    stages = ctx.timing()
    ctx.set_timing(False)
    ctx.close()
    return dict(ms_per_step=1000.0 * wall / steps, gpu_ms_per_step=gpu_ms / steps, nll=out[0],
                grad=None if out[1] is None else [float(v) for v in out[1]],
                stages={k: v[0] / max(v[1], 1) for k, v in stages.items() if v[1] > 0})


def estimate_leg(w, Xd, Zd, yd, precision="fp32"):
    """L-BFGS estimation of (sigma1^2, range, s2) at C2 from a perturbed start,
    every evaluation on the GPU, neighbours re-selected at power-of-two
    iterations and at convergence (one whole estimation, timed once)."""
    import torch
    from paper_2507_05064_amd.estimate import estimate_gaussian
    from paper_2507_05064_amd.vif import VifContext
    ctx = VifContext(w.n, w.d, w.m, w.m_v, kernel=w.kernel, likelihood=w.likelihood, precision=precision,
                     tau_m=w.tau_m)
    theta0 = w.theta * np.array([1.5, 0.7, 2.0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = estimate_gaussian(ctx, Xd, Zd, yd, theta0, reselect=True)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    ctx.close()
    return {"seconds": sec, "theta0": [float(v) for v in theta0], "theta_hat": [float(v) for v in res["theta"]],
            "theta_true": [float(v) for v in w.theta], "nll": res["nll"], "iterations": res["iterations"],
            "evaluations": res["evaluations"], "reselections": res["reselections"], "restarts": res["restarts"],
            "lbfgs_message": res["message"], "form": precision}


def predict_leg(w, Xd, Zd, nbr, yd, n_pred=100_000, reps=5):
    """Prediction at C2 (Prop. 2.1, B_p = I) at n_pred seeded uniform points:
    the prediction-neighbour search once, then the predictive mean alone and
    mean plus variances (median of reps calls after one warm-up), FP64 and
    FP32 forms on the same neighbour sets; the FP32 results against FP64's."""
    import torch
    import vif_inputs as vi
    from paper_2507_05064_amd.vif import VifContext
    Xp = torch.from_numpy(vi.coords(vi.scaled(w, n_pred), 1)).to("cuda")
    out, res = {}, {}
    for prec in ("fp64", "fp32"):
        ctx = VifContext(w.n, w.d, w.m, w.m_v, kernel=w.kernel, likelihood=w.likelihood, precision=prec,
                         tau_m=w.tau_m, max_pred=n_pred)
        ctx.build_factor(Xd, Zd, nbr, w.theta)
        if prec == "fp64":
            ctx.select_neighbors_pred(Xp)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nbrp = ctx.select_neighbors_pred(Xp)
            torch.cuda.synchronize()
            out["neighbour_search_s"] = time.perf_counter() - t0
        times = {"mean": [], "mean_var": []}
        for r in range(reps + 1):
            for key in times:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                got = ctx.predict(yd, Xp, nbrp, variances=(key == "mean_var"))
                torch.cuda.synchronize()
                if r:
                    times[key].append(time.perf_counter() - t0)
        mu, var = got
        res[prec] = (mu.cpu().numpy(), var.cpu().numpy())
        out[prec] = {"mean_ms": 1e3 * float(np.median(times["mean"])),
                     "mean_var_ms": 1e3 * float(np.median(times["mean_var"])),
                     "points_per_s_mean_var": n_pred / float(np.median(times["mean_var"]))}
        ctx.close()
    (m64, v64), (m32, v32) = res["fp64"], res["fp32"]
    out.update({"n_pred": n_pred, "var_min": float(v64.min()), "var_max": float(v64.max()),
                "fp32_mean_rel_diff": float(np.max(np.abs(m32 - m64)) / np.max(np.abs(m64))),
                "fp32_var_rel_diff": float(np.max(np.abs(v32 - v64)) / np.max(v64))})
    return out


def _pct(v, q):
    return float(np.percentile(np.asarray(v), q))


def pcg_leg(reps, log):
    """Only the C3 mode solves from zero (VIFDU and FITC), for kernel traces
    and counters of the solve kernels: no network, no prediction, no SLQ."""
    import torch
    import vif_inputs as vi
    from paper_2507_05064_amd import warmstart as ws
    prob = ws.make_problem(vi.config3(), 0)
    ctx = ws.context_for(prob, cg_tol=1e-6)
    ctx.build_factor(prob.X, prob.Z, prob.nbr, prob.theta)
    out = {}
    for form in ("vifdu", "fitc"):
        ctx.set_preconditioner(form)
        ms = []
        for r in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st, _ = ctx.laplace_mode(prob.y)
            torch.cuda.synchronize()
            if r > 0:
                ms.append(1000.0 * (time.perf_counter() - t0))
        out[form] = {"mode_ms_median": _pct(ms, 50), "pcg_iters_total": st["pcg_iters_total"],
                     "newton_iters": st["newton_iters"]}
        log(f"pcg {form}: {out[form]}")
    ctx.close()
    return out


def laplace_leg(reps, warmup, log):
    """Mode time and iterations, zero start vs learned warm start (FP64)."""
    import torch
    import vif_inputs as vi
    from paper_2507_05064_amd import warmstart as ws
    w = vi.config3()
    t0 = time.perf_counter()
    train = [ws.make_problem(w, p, theta_scale=sc) for p, sc in ((11, (0.8, 1.1)), (12, (1.25, 0.9)), (13, (1.0, 1.0)))]
    feat, target = ws.training_pairs(train, cg_tol=1e-8)
    del train
    log(f"laplace: {feat.shape[0]} training pairs in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    mlp = ws.train(feat, target, epochs=20)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del feat, target
    prob = ws.make_problem(w, 0)
    ctx = ws.context_for(prob, cg_tol=1e-6, max_pred=50_000, max_probes=16)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    build_ms = []
    for r in range(warmup + reps):
        ev[0].record()
        ctx.build_factor(prob.X, prob.Z, prob.nbr, prob.theta)
        ev[1].record()
        torch.cuda.synchronize()
        if r >= warmup:
            build_ms.append(ev[0].elapsed_time(ev[1]))
    out = {}
    modes = {}
    # VIFDU (eq. pcls1) from zero and from the learned start, then the same
    # with the FITC preconditioner (eq. pcls2)
    for form in ("zero", "warm", "fitc_zero", "fitc_warm"):
        ctx.set_preconditioner("fitc" if form.startswith("fitc") else "vifdu")
        ms, st = [], None
        for r in range(warmup + reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if form.endswith("zero"):
                mode, st, _ = ctx.laplace_mode(prob.y)
            else:
                b0 = mlp.forward(ctx.mlp_features(prob.y), double=True)
                mode, st, _ = ctx.laplace_mode(prob.y, b0)
            torch.cuda.synchronize()
            if r >= warmup:
                ms.append(1000.0 * (time.perf_counter() - t0))
        modes[form] = mode
        out[form] = {"mode_ms_median": _pct(ms, 50), "mode_ms_p10": _pct(ms, 10), "mode_ms_p90": _pct(ms, 90),
                     "newton_iters": st["newton_iters"], "pcg_iters_total": st["pcg_iters_total"],
                     "pcg_iters": st["pcg_iters"], "halvings": st["halvings"], "start_used": st["start_used"],
                     "psi": st["psi"], "levels_fwd": st["levels_fwd"], "levels_bwd": st["levels_bwd"],
                     "wide_fwd": st["wide_fwd"], "wide_bwd": st["wide_bwd"]}
        if form.endswith("zero"):
            # one more solve with per-stage HIP events (outside the timed
            # reps: the events synchronise at the end of every PCG solve)
            ctx.set_timing(True)
            _, st_t, _ = ctx.laplace_mode(prob.y)
            tm = ctx.timing()
            ctx.set_timing(False)
            pcg_ms, _ = tm["laplace_pcg"]
            out[form]["pcg_ms_total"] = pcg_ms
            out[form]["pcg_ms_per_iter"] = pcg_ms / max(st_t["pcg_iters_total"], 1)
        log(f"laplace {form}: {out[form]}")
    b0 = mlp.forward(ctx.mlp_features(prob.y), double=True)
    ref = modes["zero"]
    out["net_rel_err"] = float(torch.linalg.norm(b0 - ref) / torch.linalg.norm(ref))
    out["mode_rel_diff"] = float(torch.linalg.norm(modes["warm"] - ref) / torch.linalg.norm(ref))
    out["speedup_warm_vs_zero"] = out["zero"]["mode_ms_median"] / out["warm"]["mode_ms_median"]
    out["fitc_mode_rel_diff_vs_vifdu"] = float(torch.linalg.norm(modes["fitc_zero"] - ref) / torch.linalg.norm(ref))
    out["fitc_speedup_warm_vs_zero"] = out["fitc_zero"]["mode_ms_median"] / out["fitc_warm"]["mode_ms_median"]
    out["factor_build_ms_median"] = _pct(build_ms, 50)
    it_bytes = pcg_iter_bytes(w.n, w.m, w.m_v)
    it_ms = out["zero"]["pcg_ms_per_iter"]
    ach = it_bytes / (it_ms * 1e-3) / 1e9
    out["roofline"] = {"bound": "hbm", "kernel": "one VIFDU-preconditioned CG iteration (all its kernels)",
                       "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                       "traffic": None, "bytes_per_iter": it_bytes, "ms_per_iter": it_ms,
                       "timing": "HIP events around each Newton step's CG solve on the library stream, "
                                 "summed over one mode solve from zero, divided by its CG iterations"}
    out["mlp_train_s"] = train_s
    # latent prediction at the mode (Prop. 3.1): omega_p and diag(Omega_p) by
    # simulation (SBPV) with 10 samples at 50000 seeded uniform points
    n_pred, ell = 50_000, 10
    Xp = torch.from_numpy(vi.coords(vi.scaled(w, n_pred), 2)).to("cuda")
    nbrp = ctx.select_neighbors_pred(Xp)
    g = torch.Generator(device="cuda").manual_seed(5)
    eps_n = torch.randn((2 * ell, w.n), dtype=torch.float64, device="cuda", generator=g)
    eps_m = torch.randn((ell, w.m), dtype=torch.float64, device="cuda", generator=g)
    ctx.set_preconditioner("vifdu")
    ctx.laplace_predict(prob.y, ref, Xp, nbrp, eps_n[:2], eps_m[:1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, var, its = ctx.laplace_predict(prob.y, ref, Xp, nbrp, eps_n, eps_m)
    torch.cuda.synchronize()
    out["predict_sbpv"] = {"n_pred": n_pred, "samples": ell, "seconds": time.perf_counter() - t0,
                           "cg_iters_total": its, "var_min": float(var.min()), "var_max": float(var.max())}
    log(f"laplace predict: {out['predict_sbpv']}")
    out["slq_compare"] = slq_compare(ctx, prob, ref, log)
    out["reps"] = reps
    out["workload"] = (f"Bernoulli-logit latent VIF: n={w.n} d={w.d} ARD Gaussian (var 1, length scales "
                       f"0.2..0.6), m={w.m} kMeans++ inducing points, m_v={w.m_v}, b from the VIF prior, "
                       f"Newton + PCG (tol 1e-6) with the VIFDU (zero, warm) or FITC (fitc_*) preconditioner, FP64")
    ctx.close()
    return out


def slq_compare(ctx, prob, mode, log, ell=8, reps=8):
    """The SLQ estimate of the Laplace NLL at the mode with the VIFDU (eq.
    slq_v1) and the FITC (eq. slq_v2) preconditioner: `reps` independent
    sets of `ell` probes, the same standard normals for both; the spread of
    the estimates over the sets (the estimator's standard deviation) and the
    time per NLL evaluation."""
    import torch
    w = prob.w
    g = torch.Generator(device="cuda").manual_seed(17)
    draws = [(torch.randn((2 * ell, w.n), dtype=torch.float64, device="cuda", generator=g),
              torch.randn((ell, w.m), dtype=torch.float64, device="cuda", generator=g)) for _ in range(reps)]
    out = {"probes": ell, "sets": reps}
    for pre in ("vifdu", "fitc"):
        ctx.set_preconditioner(pre)
        vals, ms = [], []
        for en, em in draws:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nll, _ = ctx.laplace_nll(prob.y, mode, en, em)
            torch.cuda.synchronize()
            ms.append(1000.0 * (time.perf_counter() - t0))
            vals.append(nll)
        out[pre] = {"nll_mean": float(np.mean(vals)), "nll_std": float(np.std(vals, ddof=1)),
                    "ms_median": _pct(ms, 50)}
    ctx.set_preconditioner("vifdu")
    out["std_ratio_vifdu_over_fitc"] = out["vifdu"]["nll_std"] / max(out["fitc"]["nll_std"], 1e-300)
    log(f"laplace SLQ comparison: {out}")
    return out


def batch_leg(steps, warmup, log):
    """64 independent Gaussian problems (n uniform in [5000, 50000], d = 2,
    Matern-3/2 with per-problem range in [0.02, 0.2], nugget 0.05, m = 100
    random-subset inducing points, m_v = 15), y from each problem's VIF prior:
    one vif_batch_nll_grad call = all 64 factor builds, NLLs and gradients.
    Neighbours are selected per problem before the timed region."""
    import torch
    import vif_inputs as vi
    from paper_2507_05064_amd.vif import VifBatch, VifContext
    ws = vi.config4_problems(64)
    Xs, Zs, nbrs, ys, thetas = [], [], [], [], []
    t0 = time.perf_counter()
    for p, w in enumerate(ws):
        X = vi.coords(w, p)
        Z = vi.inducing_points(w, X, p)
        Xd, Zd = torch.as_tensor(X, device="cuda"), torch.as_tensor(Z, device="cuda")
        ctx = VifContext(w.n, w.d, w.m, w.m_v, kernel=w.kernel, precision="fp64", tau_m=w.tau_m)
        nbr = ctx.select_neighbors(Xd, Zd, w.theta)
        ctx.build_factor(Xd, Zd, nbr, w.theta)
        eps1, eps2, _ = vi.prior_noise(w, p)
        y = ctx.sample_prior(torch.as_tensor(eps1, device="cuda"), torch.as_tensor(eps2, device="cuda"))
        ctx.close()
        Xs.append(Xd)
        Zs.append(Zd)
        nbrs.append(nbr)
        ys.append(y)
        thetas.append(w.theta)
    Xc, Zc, nc, yc = torch.cat(Xs), torch.cat(Zs), torch.cat(nbrs), torch.cat(ys)
    theta = np.stack(thetas)
    sizes = [w.n for w in ws]
    log(f"batch: 64 problems, {sum(sizes)} points, inputs in {time.perf_counter() - t0:.1f} s")
    out = {"workload": "64 Gaussian VIF problems, n uniform in [5000, 50000] (total %d), d=2, Matern-3/2 "
                       "(var 1, range uniform in [0.02, 0.2]), nugget 0.05, m=100 random-subset inducing points, "
                       "m_v=15, y from the VIF prior; NLL + gradient of all 64 per call" % sum(sizes),
           "problems": 64, "points": int(sum(sizes))}
    for prec in ("fp32", "fp64"):
        bt = VifBatch(sizes, 2, 100, 15, precision=prec)
        for _ in range(warmup):
            bt.nll_grad(Xc, Zc, nc, theta, yc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            nll, g = bt.nll_grad(Xc, Zc, nc, theta, yc)
        torch.cuda.synchronize()
        ms = 1000.0 * (time.perf_counter() - t0) / steps
        bt.close()
        out[prec] = {"ms_per_call": ms, "problems_per_s": 64 * 1000.0 / ms,
                     "points_per_s": sum(sizes) * 1000.0 / ms, "nll_sum": float(np.sum(nll))}
        log(f"batch {prec}: {out[prec]}")
    return out


def c5_leg(reps, log, ell=50):
    """Poisson-log latent VIF at n = 1,000,000 in [0,1]^2 (Matern-1/2, variance
    1, range 0.05, m = 500 k-means++ inducing points selected on the GPU,
    m_v = 20), FP32 factor with FP64 L_m and log-determinants. A warm-start
    network is trained on two problems drawn on the same inputs (parameters
    scaled, other prior draws), with modes by the method. One evaluation: the
    factor build, the mode from the network's start (features and network
    included), then the Laplace NLL and its gradient with ell = 50 SLQ/STE
    probes. The warm-up pass also times the mode from zero (FITC and VIFDU)."""
    import torch
    import vif_inputs as vi
    from paper_2507_05064_amd import warmstart as ws
    from paper_2507_05064_amd.vif import VifContext
    w = vi.config5()
    t0 = time.perf_counter()
    X = vi.coords(w)
    Xd = torch.as_tensor(X, device="cuda")
    ctx = VifContext(w.n, w.d, w.m, w.m_v, kernel=w.kernel, likelihood=w.likelihood, precision="fp32",
                     tau_m=w.tau_m, cg_tol=1e-6, cg_maxit=2000, max_probes=ell)
    unif = vi.rng(w.config, vi.STREAM_INDUCING, 0).uniform(size=w.m)
    Zd = ctx.select_inducing(Xd, w.theta, unif=unif, lloyd_iters=10)
    torch.cuda.synchronize()
    t_ind = time.perf_counter() - t0
    t1 = time.perf_counter()
    nbr = ctx.select_neighbors(Xd, Zd, w.theta)
    torch.cuda.synchronize()
    t_knn = time.perf_counter() - t1
    ctx.set_preconditioner("fitc")  # mode finding on eq. pcls2 with FITC

    def draw(problem, theta):
        ctx.build_factor(Xd, Zd, nbr, theta)
        eps1, eps2, u = vi.prior_noise(w, problem)
        b = ctx.sample_prior(torch.as_tensor(eps1, device="cuda"), torch.as_tensor(eps2, device="cuda"))
        return torch.as_tensor(vi.poisson_from_uniform(np.exp(b.cpu().numpy()), u), device="cuda")

    # warm-start network: training pairs from two problems on the same inputs
    t1 = time.perf_counter()
    feats, targets = [], []
    for prob, sc in ((1, (0.8, 1.1)), (2, (1.25, 0.9))):
        th = w.theta.copy()
        th[0] *= sc[0]
        th[1:-1] *= sc[1]
        y_t = draw(prob, th)
        mode_t, _, _ = ctx.laplace_mode(y_t)
        feats.append(ctx.mlp_features(y_t))
        targets.append(mode_t.float())
    mlp = ws.train(torch.cat(feats), torch.cat(targets), epochs=10)
    del feats, targets
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    yd = draw(0, w.theta)
    e3, e1, e2 = vi.probe_normals(w, ell)
    eps_n = np.empty((2 * ell, w.n))
    eps_n[0::2], eps_n[1::2] = e1.T, e2.T
    eps_nd, eps_md = torch.as_tensor(eps_n, device="cuda"), torch.as_tensor(np.ascontiguousarray(e3.T), device="cuda")
    del eps_n
    log(f"c5: inputs {time.perf_counter() - t0:.1f} s (inducing points {t_ind:.1f} s, neighbours {t_knn:.1f} s, "
        f"warm-start training {t_train:.1f} s)")
    times = {"build": [], "mode": [], "nll_grad": []}
    out = None
    zero = {}
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.build_factor(Xd, Zd, nbr, w.theta)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        b0 = mlp.forward(ctx.mlp_features(yd), double=True)
        mode, st, _ = ctx.laplace_mode(yd, b0)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ctx.set_preconditioner("vifdu")  # the gradient's trace estimates on VIFDU block solves (eq. slq_v1)
        nll, grad = ctx.laplace_nll_grad(yd, mode, eps_nd, eps_md)
        ctx.set_preconditioner("fitc")
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        if r == 0:  # the warm-up pass also times the modes from zero
            for form in ("vifdu", "fitc"):
                ctx.set_preconditioner(form)
                tv = time.perf_counter()
                mode0, stz, _ = ctx.laplace_mode(yd)
                torch.cuda.synchronize()
                zero[form] = {"mode_ms": 1000 * (time.perf_counter() - tv), "newton_iters": stz["newton_iters"],
                              "pcg_iters_total": stz["pcg_iters_total"], "psi": stz["psi"]}
            # the same NLL + gradient with the FITC preconditioner (eq. slq_v2, App. E.2)
            tv = time.perf_counter()
            nll_f, grad_f = ctx.laplace_nll_grad(yd, mode, eps_nd, eps_md)
            torch.cuda.synchronize()
            zero["fitc_nll_grad"] = {"ms": 1000 * (time.perf_counter() - tv), "nll": nll_f,
                                     "grad": [float(v) for v in grad_f]}
        if r > 0:  # the first pass warms up
            times["build"].append(1000 * (t1 - t0))
            times["mode"].append(1000 * (t2 - t1))
            times["nll_grad"].append(1000 * (t3 - t2))
        out = dict(nll=nll, grad=[float(v) for v in grad], newton_iters=st["newton_iters"],
                   pcg_iters_total=st["pcg_iters_total"], start_used=st["start_used"],
                   levels_fwd=st["levels_fwd"],
                   net_rel_err=float(torch.linalg.norm(b0 - mode) / torch.linalg.norm(mode)),
                   mode_rel_diff_vs_zero_start=float(torch.linalg.norm(mode - mode0) / torch.linalg.norm(mode0)),
                   psi=st["psi"])
        log(f"c5 rep {r}: build {1000 * (t1 - t0):.1f} ms, mode {1000 * (t2 - t1):.1f} ms, "
            f"nll+grad {1000 * (t3 - t2):.1f} ms, {out}")
    ctx.close()
    res = {k + "_ms_median": _pct(v, 50) for k, v in times.items()}
    res["eval_ms_median"] = sum(res.values())
    res.update(out)
    res["probes"] = ell
    res["mode_from_zero_warmup_pass"] = zero
    res["setup_s"] = {"inducing_points": t_ind, "neighbours": t_knn, "warm_start_training": t_train}
    res["workload"] = ("Poisson-log latent VIF: n=1000000 d=2 Matern-1/2 (var 1, range 0.05), m=500 k-means++ "
                       "inducing points, m_v=20, b from the VIF prior; FP32 factor; mode by Newton + FITC-PCG "
                       "(tol 1e-6) from the learned warm start, Laplace NLL + gradient with 50 SLQ/STE probes "
                       "(VIFDU, eq. slq_v1)")
    return res


def _oracle_c2_seconds(w, budget_points):
    from oracle import vif_oracle as vo
    import vif_inputs as vi
    X = vi.coords(w)[:budget_points]
    Z = vi.inducing_points(w, vi.coords(w))
    model = vo.Model(w.kernel, w.sigma1_sq, np.asarray(w.lengthscales, float), w.s2, w.tau_m)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, w.m_v)
    y = vi.normals(w, budget_points, stream=vi.STREAM_NOISE) * math.sqrt(w.sigma1_sq + w.s2)
    t0 = time.perf_counter()
    vo.nll_gaussian_grad(model, X, Z, nbr, y)
    return time.perf_counter() - t0


def _oracle_c3_mode(n0):
    """The oracle's Laplace mode (Newton with Jacobi-preconditioned CG) on a
    C3-shaped problem of n0 points: inputs of C3's distribution, m = 500
    k-means++ inducing points, m_v = 30, b from the latent VIF prior,
    Bernoulli responses, Newton tolerance 1e-9 as on the GPU."""
    from scipy.special import expit
    from oracle import laplace_oracle as lo
    from oracle import vif_oracle as vo
    import vif_inputs as vi
    w = vi.scaled(vi.config3(), n0)
    X = vi.coords(w)
    Z = vi.inducing_points(w, X)
    model = vo.Model(w.kernel, w.sigma1_sq, np.asarray(w.lengthscales, float), w.s2, w.tau_m)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, w.m_v)
    prior = lo.LatentVIF.build(model, X, Z, nbr)
    eps1, eps2, u = vi.prior_noise(w)
    b = vo.prior_sample(nbr, prior.fac, ind, eps1, eps2)
    y = vi.bernoulli_from_uniform(expit(b), u)

    def run():
        t0 = time.perf_counter()
        r = lo.find_mode(prior, lo.BERNOULLI_LOGIT, y, tol=1e-9, solver="cg")
        return time.perf_counter() - t0, r.iters

    return run


def cpu_baseline(w, budget_points=6000, c3_points=1500):
    """The oracle (FP64 numpy/scipy) on the host cores, with numpy's BLAS
    threads and with one thread:
      * C2: NLL + forward-mode gradient on the first `budget_points` points of
        the same workload (the prefix is itself a VIF problem: its
        conditioning sets only reach earlier points), scaled by
        n / budget_points to evaluations per second at full n;
      * C3: the oracle's Laplace mode on a C3-shaped problem of `c3_points`
        points (not scaled: its CG iteration counts depend on n)."""
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    sec = _oracle_c2_seconds(w, budget_points)
    with threadpool_limits(1):
        sec1 = _oracle_c2_seconds(w, budget_points)
    run = _oracle_c3_mode(c3_points)
    c3_sec, c3_it = run()
    with threadpool_limits(1):
        c3_sec1, _ = run()
    scale = w.n / budget_points
    return {"value": 1.0 / (sec * scale), "unit": "evals/s", "cores": int(threads), "kind": "oracle",
            "sample": f"NLL + forward-mode gradient on the first {budget_points} of {w.n} points "
                      f"({sec:.1f} s), scaled linearly to n={w.n}",
            "single_thread": {"value": 1.0 / (sec1 * scale), "unit": "evals/s", "cores": 1,
                              "sample": f"the same with one BLAS thread ({sec1:.1f} s)"},
            "c3_mode": {"seconds": c3_sec, "seconds_one_thread": c3_sec1, "newton_iters": int(c3_it),
                        "cores": int(threads), "n": c3_points,
                        "sample": f"oracle Laplace mode (Newton, Jacobi-preconditioned CG to 1e-12, Newton "
                                  f"tolerance 1e-9) on a C3-shaped problem of {c3_points} points (d=5 ARD "
                                  f"Gaussian, m=500 k-means++ inducing points, m_v=30, Bernoulli-logit); "
                                  f"not scaled to n=200000"}}


def counters_mode(w):
    """Workload for `rocprofv3 --pmc`: five factor builds and NLL + gradient
    evaluations at C2 (FP32), then five plain device copies of 1 GiB, whose
    FETCH_SIZE / WRITE_SIZE readings give the counters' scale against known
    bytes."""
    import torch
    import vif_inputs as vi
    from paper_2507_05064_amd.vif import VifContext
    X = vi.coords(w)
    Z = vi.inducing_points(w, X)
    Xd, Zd = torch.as_tensor(X, device="cuda"), torch.as_tensor(Z, device="cuda")
    ctx = VifContext(w.n, w.d, w.m, w.m_v, kernel=w.kernel, precision="fp32", tau_m=w.tau_m)
    nbr = ctx.select_neighbors(Xd, Zd, w.theta)
    y = torch.as_tensor(vi.normals(w, w.n, stream=vi.STREAM_NOISE) * math.sqrt(w.sigma1_sq + w.s2), device="cuda")
    for _ in range(5):
        ctx.build_factor(Xd, Zd, nbr, w.theta)
        ctx.nll_grad(y, w.theta.size)
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)  # 1 GiB
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"factor_bytes_per_launch": w.n * factor_bytes_per_point(w.m, w.m_v, w.d, 4),
                      "factor_bwd_bytes_per_launch": w.n * factor_bwd_bytes_per_point(w.m, w.m_v, w.d, 4),
                      "copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--nll-only", action="store_true", help="time the NLL without the gradient")
    ap.add_argument("--no-laplace", action="store_true", help="skip the Laplace mode leg")
    ap.add_argument("--laplace-reps", type=int, default=5)
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-problem batched leg")
    ap.add_argument("--counters", action="store_true",
                    help="hardware-counter mode: 5 FP32 factor builds of the C2 workload and 5 copies of a 1 GiB "
                         "buffer (the counters' scale reference), nothing timed")
    ap.add_argument("--pcg-only", action="store_true",
                    help="only the n = 200k mode solves from zero, VIFDU and FITC (for kernel traces and counters)")
    ap.add_argument("--c2-only", action="store_true",
                    help="only the n = 100k NLL + gradient step in its three forms (for kernel traces and counters)")
    ap.add_argument("--laplace-only", action="store_true",
                    help="only the n = 200k Laplace leg (for its kernel trace)")
    ap.add_argument("--skip-c5", action="store_true",
                    help="leave out the n = 1M Poisson leg (its set-up, neighbour search and warm-start training, "
                         "takes about a minute)")
    ap.add_argument("--c5-only", action="store_true", help="only the n = 1M Poisson leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import vif_inputs as vi
    from paper_2507_05064_amd.vif import VifContext

    w = vi.config2()
    if args.counters:
        counters_mode(w)
        return
    if args.laplace_only:
        print(json.dumps({"laplace": laplace_leg(args.laplace_reps, 1,
                                                 lambda msg: print(msg, file=sys.stderr, flush=True))}))
        return
    if args.c5_only:
        print(json.dumps({"laplace_nll_grad_c5": c5_leg(2, lambda msg: print(msg, file=sys.stderr, flush=True))}))
        return
    if args.pcg_only:
        print(json.dumps({"pcg": pcg_leg(args.laplace_reps, lambda msg: print(msg, file=sys.stderr, flush=True))}))
        return
    X = vi.coords(w)
    Z = vi.inducing_points(w, X)
    Xd = torch.as_tensor(X, device="cuda")
    Zd = torch.as_tensor(Z, device="cuda")
    sel = VifContext(w.n, w.d, w.m, w.m_v, kernel=w.kernel, precision="fp64", tau_m=w.tau_m)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nbr = sel.select_neighbors(Xd, Zd, w.theta)
    torch.cuda.synchronize()
    knn_s = time.perf_counter() - t0
    sel.close()
    # response: a draw from the VIF prior at the true parameters,
    # y = V^T eps1 + B^{-1} D^{1/2} eps2 with the nugget inside D
    samp = VifContext(w.n, w.d, w.m, w.m_v, kernel=w.kernel, precision="fp64", tau_m=w.tau_m)
    samp.build_factor(Xd, Zd, nbr, w.theta)
    eps1, eps2, _ = vi.prior_noise(w)
    yd = samp.sample_prior(torch.as_tensor(eps1, device="cuda"), torch.as_tensor(eps2, device="cuda"))
    samp.close()
    grad = not args.nll_only

    r32 = run_form(w, Xd, Zd, nbr, yd, "fp32", args.steps, args.warmup, grad)
    r64 = run_form(w, Xd, Zd, nbr, yd, "fp64", args.steps, args.warmup, grad)
    r16 = run_form(w, Xd, Zd, nbr, yd, "bf16_in", args.steps, args.warmup, grad)

    fac_ms = r32["stages"].get("factor", float("nan"))
    nbytes = w.n * factor_bytes_per_point(w.m, w.m_v, w.d, 4)
    achieved = nbytes / (fac_ms * 1e-3) / 1e9
    bwd_ms = r32["stages"].get("grad_factor_bwd", float("nan"))
    bwd_bytes = w.n * factor_bwd_bytes_per_point(w.m, w.m_v, w.d, 4)
    bwd_achieved = bwd_bytes / (bwd_ms * 1e-3) / 1e9
    nll_rel16 = abs(r16["nll"] - r64["nll"]) / abs(r64["nll"])
    grad_err16 = (None if r16["grad"] is None else
                  float(np.max(np.abs(np.subtract(r16["grad"], r64["grad"]))) / np.max(np.abs(r64["grad"]))))
    res = {
        "metric": METRIC,
        "value": 1000.0 / r32["ms_per_step"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": f"Gaussian VIF NLL{'+grad' if grad else ''}: n={w.n} d={w.d} Matern-3/2 "
                               f"(var 1, range 0.05), nugget 0.05, m={w.m} random-subset inducing points, "
                               f"m_v={w.m_v} correlation neighbours, random ordering",
                   "objective": "nll+grad" if grad else "nll", "n": w.n, "m": w.m, "m_v": w.m_v},
        "fp64": {"value": 1000.0 / r64["ms_per_step"], "unit": "evals/s", "ms_per_step": r64["ms_per_step"],
                 "nll": r64["nll"], "grad": r64["grad"]},
        "fp32_nll": r32["nll"],
        "fp32_grad": r32["grad"],
        "fp32_rel_err_vs_fp64_gpu": abs(r32["nll"] - r64["nll"]) / abs(r64["nll"]),
        "bf16_in": {"value": 1000.0 / r16["ms_per_step"], "unit": "evals/s", "ms_per_step": r16["ms_per_step"],
                    "nll": r16["nll"], "grad": r16["grad"],
                    "nll_rel_err_vs_fp64_gpu": nll_rel16,
                    "nll_err_per_point_vs_fp64_gpu": abs(r16["nll"] - r64["nll"]) / w.n,
                    "grad_err_vs_fp64_gpu": grad_err16,
                    # the BF16-input bar: NLL within 1e-3 relative, gradient within 5e-2 of max |g|
                    "within_bar": bool(nll_rel16 <= 1e-3 and (grad_err16 is None or grad_err16 <= 5e-2)),
                    "stage_ms": r16["stages"]},
        "stage_ms": {"fp32": r32["stages"], "fp64": r64["stages"]},
        "neighbour_search_s": knn_s,
        # the dominant kernel of the step: the adjoint of the per-point factor
        "roofline": {"bound": "hbm", "kernel": "k_factor_bwd<float>", "achieved": bwd_achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": bwd_achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("k_factor_bwd"), "bytes_per_launch": bwd_bytes,
                     "avg_launch_ms": bwd_ms},
        "roofline_factor": {"bound": "hbm", "kernel": "k_factor<float>", "achieved": achieved, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                            "traffic": measured_traffic("k_factor"), "bytes_per_launch": nbytes,
                            "avg_launch_ms": fac_ms},
    }
    if args.c2_only:
        print(json.dumps(res))
        return
    res["predict"] = predict_leg(w, Xd, Zd, nbr, yd)
    res["estimate"] = {"fp32": estimate_leg(w, Xd, Zd, yd, "fp32"), "fp64": estimate_leg(w, Xd, Zd, yd, "fp64")}
    if not args.no_batch:
        res["batch"] = batch_leg(args.steps, args.warmup, lambda msg: print(msg, file=sys.stderr, flush=True))
    if not args.no_laplace:
        res["laplace"] = laplace_leg(args.laplace_reps, 1, lambda msg: print(msg, file=sys.stderr, flush=True))
    if not args.skip_c5:
        res["laplace_nll_grad_c5"] = c5_leg(2, lambda msg: print(msg, file=sys.stderr, flush=True))
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
