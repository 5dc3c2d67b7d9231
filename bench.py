#!/usr/bin/env python3
"""Benchmark of the self-learning DQMC hot path on one MI355X.

Headline workload: the learned-action workload's lattice, 48x48 (N = 2304
sites), L = 100 slices (beta = 10, dtau = 0.1), t = 1, mu = -0.5, xi = 1.5, QR
stabilisation every 10 slices, FP64 judge.  A batch of B independent chains
(256 by default: 65 GB of the 288 GB) starts from seeded iid +-1 fields; the
linear effective action (1 + 2 + 50 + 4 = 57 terms) is fitted on the GPU to
their exact weights.

One timed step = one cumulative update (steps iii-iv of the method, Eq. 4) of
every chain: one sweep of colour-class effective moves (N L = 230 400
single-flip proposals), the exact weight of the proposal (10 blocks of 10
structured slice products, 10 QR stabilisations, the final determinant) and
the accept/reject.  Each step therefore makes exactly B exact fermion-weight
evaluations, and value = B * steps / seconds.

The roofline object is that of the stabilisation, the part of an evaluation
that takes most of its time: algorithmic flops of the QRs with their explicit
Q and of the V updates, over the HIP-event time of those launch sequences on
the call's stream in the timed region.  The chain products (the structured
FP64 slice products) and the final determinant are reported beside it.
cpu_baseline times the oracle on one chain of the same workload (one
cumulative update with all host threads; one with one thread on the same
lattice with 20 slices, scaled by 5 to 100).

Other reports, each printing its own JSON line: --workload dqmc_20x20 (the
20x20, L = 80 workload as the headline), --sweeps-only (local DQMC sweeps),
--ess-only (effective samples per second of the self-learning procedure
against FP64 DQMC), --reports (uneven groups, precision modes, learned
proposals).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "exact fermion-weight evals/sec + effective indep. samples/sec vs FP64 DQMC"
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 matrix (and vector) peak
COPY_CALIBRATION_BYTES = 1 << 30
# HBM bytes per stabilisation (all launches of one QR with its explicit Q and
# V update, over the batch), by (workload, batch): rocprofv3 --pmc
# FETCH_SIZE, then WRITE_SIZE, summed over the stabilisation kernels of an
# evaluation, divided by its 10 stabilisations, each scaled by what the same
# counter reads for the 1 GiB copy of --copy-calibration (FETCH_SIZE reads
# half of the copied bytes, WRITE_SIZE all of them).
STAB_TRAFFIC = {("learned_48x48", 256): 5.38444e11 + 1.48524e11}


def oracle_cumulative_step_seconds(model, terms, theta, field, threads, seed):
    """Seconds of one oracle cumulative update (one effective sweep and one
    exact weight) of one chain, with `threads` BLAS threads (None: all)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import effective, stable
    c0, lam = float(theta[0]), np.asarray(theta[1:], dtype=np.float64)
    classes = effective.colour_classes(model, terms)
    with threadpool_limits(limits=threads):
        la, sg = stable.weight(model, field)      # the incoming weight (not timed)
        t0 = time.perf_counter()
        effective.cumulative_step(model, terms, c0, lam, field.copy(), la, sg, len(classes),
                                  lambda x: stable.weight(model, x), seed=seed, step=0, classes=classes)
        return time.perf_counter() - t0


def cpu_baseline(model, terms, theta, field, seed):
    """The oracle's cumulative update on one chain, timed on the host cores:
    all threads on the full workload; one thread on the same lattice with L
    reduced to 20 (one fifth of the slices, so of the chain products and
    stabilisations; the effective sweep is one fifth as long too), scaled by 5."""
    from threadpoolctl import threadpool_info
    cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [os.cpu_count() or 1])
    t_all = oracle_cumulative_step_seconds(model, terms, theta, field, None, seed)
    short = model.with_(n_slices=20)
    from slq_inputs import default_terms, iid_field
    t_one = oracle_cumulative_step_seconds(short, default_terms(20), [theta[0]] + [0.0] * len(default_terms(20)),
                                           iid_field(short, 2100), 1, seed) * (model.n_slices / 20)
    return {"value": 1.0 / t_all, "unit": "evals/s", "cores": int(cores), "kind": "oracle",
            "sample": f"one cumulative update of one chain at {model.lx}x{model.ly}, L={model.n_slices} "
                      f"({t_all:.1f} s: one effective sweep of N L proposals and one exact weight, "
                      f"NumPy/SciPy FP64 with {cores} BLAS threads)",
            "one_thread": {"value": 1.0 / t_one, "cores": 1,
                           "sample": f"one cumulative update at {model.lx}x{model.ly}, L=20, one BLAS thread, "
                                     f"scaled by {model.n_slices // 20} to L={model.n_slices} ({t_one:.1f} s)"}}


def ess_rates(slq, plan, model, terms, seed, steps, n, sweeps, burn):
    """Effective independent samples per second of the total magnetisation M,
    following the self-learning procedure with n chains on both sides:
    (i) local FP64 DQMC sweeps (timed), whose configurations and exact weights
    form the training set; (ii) the effective model fitted to them;
    (iii)+(iv) cumulative updates started from the DQMC end configurations,
    for a few numbers of effective moves per update, with the FP64 judge, with
    FP32 chain products in the judge, and with proposals from a network action
    trained on the residual of the fit.  An ESS ratio is quoted only where
    the two samplers agree on <M>, <M^2> and <sign> within 2 standard errors
    (equal accuracy); tau_int is not clamped."""
    import numpy as np
    import torch
    from paper_1612_03804_amd.analysis import tau_int_chains, mean_and_error, agree
    from slq_inputs import iid_fields, net_init
    dev = torch.device("cuda")
    L, N = model.n_slices, model.n_sites
    f64, i8, i32, i64 = torch.float64, torch.int8, torch.int32, torch.int64
    s_dq = torch.from_numpy(iid_fields(model, n, 3000)).to(dev)
    G = torch.empty((n, N, N), dtype=f64, device=dev)
    la = torch.empty(n, dtype=f64, device=dev)
    sg = torch.empty(n, dtype=i8, device=dev)
    st = torch.empty(n, dtype=i32, device=dev)
    a64 = torch.empty(n, dtype=i64, device=dev)
    drift = torch.empty(n, dtype=f64, device=dev)
    slq.slq_green(plan, s_dq, G, la, sg, st)
    slq.slq_sweep_local(plan, s_dq, G, la, sg, burn, seed, 0, 0, a64, drift, st)
    keep = max(1, sweeps // 50)           # every keep-th configuration goes to the training set
    train_s = torch.empty((sweeps // keep, n, L, N), dtype=i8, device=dev)
    train_la = torch.empty((sweeps // keep, n), dtype=f64, device=dev)
    Md = torch.empty((sweeps, n), dtype=i64, device=dev)
    Sd = torch.empty((sweeps, n), dtype=i8, device=dev)
    acc_dq = torch.zeros(n, dtype=i64, device=dev)
    max_drift = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(sweeps):
        slq.slq_sweep_local(plan, s_dq, G, la, sg, 1, seed, 1000 + k, 0, a64, drift, st)
        slq.slq_magnetization(plan, s_dq, Md[k])
        Sd[k].copy_(sg)
        if k % keep == 0 and k // keep < train_s.shape[0]:
            train_s[k // keep].copy_(s_dq)
            train_la[k // keep].copy_(la)
        acc_dq += a64
    torch.cuda.synchronize()
    t_dq = time.perf_counter() - t0
    max_drift = float(drift.max().item())
    Mh, Sh = Md.cpu().numpy().T.astype(np.float64), Sd.cpu().numpy().T.astype(np.float64)
    tau_dq = tau_int_chains(Mh)
    obs_dq = {"M": mean_and_error(Mh), "M2": mean_and_error(Mh ** 2), "sign": mean_and_error(Sh)}
    dq = {"chains": n, "sweeps": sweeps, "sweeps_per_s": n * sweeps / t_dq, "tau_int_sweeps": tau_dq,
          "ess_per_s": n * sweeps / (2 * tau_dq) / t_dq if tau_dq > 0 else None,
          "local_acceptance": float(acc_dq.sum().item()) / (n * sweeps * N * L), "max_drift": max_drift,
          "observables": obs_dq}

    # (ii) fit on the DQMC configurations
    eff = slq.Eff(plan, terms, np.zeros(len(terms)))
    theta = torch.empty(1 + len(terms), dtype=f64, device=dev)
    r2 = torch.empty(1, dtype=f64, device=dev)
    xs, ys = train_s.view(-1, L, N), train_la.view(-1)
    slq.slq_fit_effective(plan, eff, xs, ys, theta, r2)
    slq.slq_eff_set_theta(eff, theta)
    start = s_dq.clone()

    def cumulative_run(pl, ef, n_moves):
        s = start.clone()
        logabs = torch.empty(n, dtype=f64, device=dev)
        sign = torch.empty(n, dtype=i8, device=dev)
        status = torch.empty(n, dtype=i32, device=dev)
        slq.slq_weight(pl, s, logabs, sign, status)
        acc = torch.empty((steps, n), dtype=i8, device=dev)
        logA = torch.empty((steps, n), dtype=f64, device=dev)
        M = torch.empty((steps, n), dtype=i64, device=dev)
        S = torch.empty((steps, n), dtype=i8, device=dev)
        for k in range(burn):
            slq.slq_cumulative_step(pl, ef, s, logabs, sign, n_moves, seed, 10_000 + k, 0, acc[0], logA[0], status)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            slq.slq_cumulative_step(pl, ef, s, logabs, sign, n_moves, seed, 20_000 + k, 0, acc[k], logA[k], status)
            slq.slq_magnetization(pl, s, M[k])
            S[k].copy_(sign)
        torch.cuda.synchronize()
        t_sl = time.perf_counter() - t0
        rate = float(acc.float().mean().item())
        la_h = logA.cpu().numpy()
        Mh2, Sh2 = M.cpu().numpy().T.astype(np.float64), S.cpu().numpy().T.astype(np.float64)
        obs = {"M": mean_and_error(Mh2), "M2": mean_and_error(Mh2 ** 2), "sign": mean_and_error(Sh2)}
        same = all(agree(obs[k], obs_dq[k]) for k in obs)
        tau_sl = tau_int_chains(Mh2) if rate > 0 else None
        ess = n * steps / (2 * tau_sl) / t_sl if tau_sl and tau_sl > 0 else None
        return {"effective_moves": n_moves, "acceptance": rate, "logA_mean": float(la_h.mean()),
                "logA_std": float(la_h.std()), "steps_per_s": n * steps / t_sl, "tau_int_steps": tau_sl,
                "ess_per_s": ess, "observables": obs, "agrees_with_dqmc_2sigma": same,
                "ess_ratio_vs_dqmc": (ess / dq["ess_per_s"]) if (same and ess and dq["ess_per_s"]) else None}, s

    runs = [cumulative_run(plan, eff, m)[0] for m in (max(1, eff.n_classes // 4), eff.n_classes, 4 * eff.n_classes)]
    best = max(runs, key=lambda r: r["ess_per_s"] or 0.0)
    n_best = best["effective_moves"]

    # FP32 chain products in the judge; its error measured on the fields it sampled
    plan32 = slq.Plan(model, n, chain_prec=slq.SLQ_PREC_FP32)
    eff32 = slq.Eff(plan32, terms, np.zeros(len(terms)))
    slq.slq_eff_set_theta(eff32, theta)
    run32, s32 = cumulative_run(plan32, eff32, n_best)
    la64 = torch.empty(n, dtype=f64, device=dev)
    la32 = torch.empty(n, dtype=f64, device=dev)
    sg_w = torch.empty(n, dtype=i8, device=dev)
    st_w = torch.empty(n, dtype=i32, device=dev)
    slq.slq_weight(plan, s32, la64, sg_w, st_w)
    slq.slq_weight(plan32, s32, la32, sg_w, st_w)
    run32["max_rel_dlogW_vs_fp64"] = float(((la32 - la64).abs() / la64.abs().clamp(min=1.0)).max().item())
    eff32.close()
    plan32.close()

    # learned action: network (FP32 training kernels, Adam) on the residual of
    # the linear fit, 90 % train / 10 % held out, output layer started at zero;
    # proposals from the best epoch if it beats the linear model on held-out
    # fields, else the linear fallback; moves and Eq. 4 in FP64
    n_all = xs.shape[0]
    n_tr = n_all - n_all // 10
    prm = torch.from_numpy(net_init(seed)).to(dev)
    prm[1960:] = 0.0
    mom, vel, g = torch.zeros_like(prm), torch.zeros_like(prm), torch.empty_like(prm)
    loss = torch.empty(1, dtype=f64, device=dev)

    def held_out(params):
        tot = 0.0
        for k in range(n_tr, n_all, n):
            e = min(n_all, k + n)
            slq.slq_net_gradient(plan, eff, slq.SLQ_PREC_FP32, xs[k:e].contiguous(), ys[k:e].contiguous(), params,
                                 g, loss)
            tot += float(loss.item()) * (e - k) / (n_all - n_tr)
        return tot

    mse_lin = held_out(torch.zeros_like(prm))
    best_prm, best_mse, curve = None, mse_lin, []
    order = np.random.default_rng(seed)
    t_adam, batch, epochs = 0, 64, 6
    t0 = time.perf_counter()
    for _ in range(epochs):
        perm = torch.from_numpy(order.permutation(n_tr)).to(dev)
        for k in range(0, n_tr - batch + 1, batch):
            idx = perm[k:k + batch]
            slq.slq_net_gradient(plan, eff, slq.SLQ_PREC_FP32, xs[idx].contiguous(), ys[idx].contiguous(), prm, g,
                                 loss)
            t_adam += 1
            slq.slq_net_adam(prm, g, mom, vel, t_adam, lr=1e-3)
        curve.append(held_out(prm))
        if curve[-1] < best_mse:
            best_mse, best_prm = curve[-1], prm.clone()
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    if best_prm is not None:
        slq.slq_eff_set_net(eff, best_prm, slq.SLQ_PREC_FP64)
    run_net, _ = cumulative_run(plan, eff, n_best)
    run_net["training"] = {"samples": n_tr, "held_out": n_all - n_tr, "epochs": epochs, "adam_steps": t_adam,
                           "seconds": t_train, "held_out_mse_linear": mse_lin, "held_out_mse_by_epoch": curve,
                           "proposals_from": "linear + network" if best_prm is not None else
                           "linear (fallback: no epoch beat the linear model on held-out fields)"}
    slq.slq_eff_set_net(eff, None)
    eff.close()
    return {"workload": "dqmc_20x20", "dqmc_fp64": dq, "fit": {"samples": n_all, "terms": len(terms),
                                                               "r2": float(r2.item())},
            "sldqmc": {"chains": n, "steps": steps, "runs": runs},
            "sldqmc_fp32_chain": run32, "sldqmc_learned_action": run_net, "burn_in": burn,
            "ess_ratio": best["ess_ratio_vs_dqmc"], "ess_ratio_fp32_chain": run32["ess_ratio_vs_dqmc"],
            "ess_ratio_learned_action": run_net["ess_ratio_vs_dqmc"]}


def local_sweep_rate(slq, plan, model, sweeps, seed):
    """Local DQMC sweeps per second on all chains of the plan (one untimed
    sweep first)."""
    import torch
    from slq_inputs import iid_fields
    dev = torch.device("cuda")
    B, N = plan.max_batch, model.n_sites
    s = torch.from_numpy(iid_fields(model, B, 3000)).to(dev)
    G = torch.empty((B, N, N), dtype=torch.float64, device=dev)
    la = torch.empty(B, dtype=torch.float64, device=dev)
    sg = torch.empty(B, dtype=torch.int8, device=dev)
    st = torch.empty(B, dtype=torch.int32, device=dev)
    acc = torch.empty(B, dtype=torch.int64, device=dev)
    drift = torch.empty(B, dtype=torch.float64, device=dev)
    slq.slq_green(plan, s, G, la, sg, st)
    slq.slq_sweep_local(plan, s, G, la, sg, 1, seed, 0, 0, acc, drift, st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    slq.slq_sweep_local(plan, s, G, la, sg, sweeps, seed, 1, 0, acc, drift, st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"mode": "local_sweeps", "workload": "dqmc_20x20", "chains": B, "sweeps": sweeps,
            "sweeps_per_s": B * sweeps / dt, "acceptance": float(acc.sum().item()) / (B * sweeps * N * model.n_slices),
            "max_drift": float(drift.max().item())}


PRECISION_PEAK_TFLOPS = {0: 78.6, 3: 78.6, 1: 157.3, 2: 2500.0}  # FP64 vector / FP64, FP32, BF16 dense MFMA


def learned_48x48_rates(slq, fields: int = 64):
    """The largest workload, 48x48 (N = 2304), L = 100: exact weights per
    second of `fields` fields, and cumulative updates per second of the same
    chains with N L single-flip proposals each (one effective sweep), proposed
    by the linear action and by the linear action plus the network (FP32, its
    output layer at zero so the proposals are those of the linear part; the
    network's forward passes and flip differences are all computed)."""
    import numpy as np
    import torch
    from slq_inputs import LEARNED_48x48, iid_fields, default_terms, net_init
    dev = torch.device("cuda")
    model = LEARNED_48x48
    F, N, L = fields, model.n_sites, model.n_slices
    plan = slq.Plan(model, F, net=True)
    slq.slq_plan_tune(plan, F)
    s = torch.from_numpy(iid_fields(model, F, 6200)).to(dev)
    la = torch.empty(F, dtype=torch.float64, device=dev)
    sg = torch.empty(F, dtype=torch.int8, device=dev)
    st = torch.empty(F, dtype=torch.int32, device=dev)
    slq.slq_weight(plan, s, la, sg, st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    slq.slq_weight(plan, s, la, sg, st)
    torch.cuda.synchronize()
    t_w = time.perf_counter() - t0
    terms = default_terms(L)
    eff = slq.Eff(plan, terms, np.zeros(len(terms)))
    acc = torch.empty(F, dtype=torch.int8, device=dev)
    logA = torch.empty(F, dtype=torch.float64, device=dev)

    def steps_per_s(n_moves, step0):
        slq.slq_cumulative_step(plan, eff, s, la, sg, n_moves, 11, step0, 0, acc, logA, st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        slq.slq_cumulative_step(plan, eff, s, la, sg, n_moves, 11, step0 + 1, 0, acc, logA, st)
        torch.cuda.synchronize()
        return F / (time.perf_counter() - t0)

    lin = steps_per_s(eff.n_classes, 0)
    prm = torch.from_numpy(net_init(12)).to(dev)
    prm[1960:] = 0.0
    slq.slq_eff_set_net(eff, prm, slq.SLQ_PREC_FP64)
    net = steps_per_s(slq.slq_eff_net_classes(eff), 10)
    S = torch.empty(F, dtype=torch.float64, device=dev)
    slq.slq_net_forward(plan, slq.SLQ_PREC_FP32, s, prm, S)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    slq.slq_net_forward(plan, slq.SLQ_PREC_FP32, s, prm, S)
    torch.cuda.synchronize()
    t_f = time.perf_counter() - t0
    ok = bool((st == 0).all().item())
    eff.close()
    plan.close()
    torch.cuda.empty_cache()
    return {"model": "48x48, L=100", "fields": F, "weights_per_s": F / t_w,
            "cumulative_steps_per_s_linear": lin, "cumulative_steps_per_s_learned": net,
            "proposals_per_step": N * L, "net_forward_samples_per_s": F / t_f, "status_ok": ok}


def learned_48x48_train(slq, chains, pairs, train_seconds, eval_steps, seed=0x5D0C + 7):
    """The learned effective action at 48x48 (N = 2304), L = 100: `pairs`
    (s, log|W_f|) pairs from `chains` chains of cumulative updates proposed by
    the linear action (one effective sweep each, after 3 burn-in updates;
    every pair's weight is the exact FP64 one the update computed), the linear
    action refitted on all of them (Eq. 3), the network trained on the GPU on
    the residual (FP32 forward and gradient kernels, Adam, batches of 64, 90 %
    train / 10 % held out, output layer started at zero, `train_seconds` of
    training), then `eval_steps` cumulative updates of the same chains
    proposed by linear + network (FP64 moves, if an epoch beat the linear
    action on held-out fields) and by the linear action alone, from the same
    start."""
    import numpy as np
    import torch
    from slq_inputs import LEARNED_48x48, iid_fields, default_terms, net_init
    dev = torch.device("cuda")
    f64, i8, i32 = torch.float64, torch.int8, torch.int32
    m = LEARNED_48x48
    C, N, L = chains, m.n_sites, m.n_slices
    plan = slq.Plan(m, C, net=True)
    slq.slq_plan_tune(plan, C)
    terms = default_terms(L)
    s = torch.from_numpy(iid_fields(m, C, 6300)).to(dev)
    la = torch.empty(C, dtype=f64, device=dev)
    sg = torch.empty(C, dtype=i8, device=dev)
    st = torch.empty(C, dtype=i32, device=dev)
    slq.slq_weight(plan, s, la, sg, st)
    eff = slq.Eff(plan, terms, np.zeros(len(terms)))
    theta = torch.empty(1 + len(terms), dtype=f64, device=dev)
    r2 = torch.empty(1, dtype=f64, device=dev)
    slq.slq_fit_effective(plan, eff, s, la, theta, r2)
    slq.slq_eff_set_theta(eff, theta)
    acc = torch.empty(C, dtype=i8, device=dev)
    logA = torch.empty(C, dtype=f64, device=dev)
    n_lin = eff.n_classes
    steps = (pairs + C - 1) // C
    xs = torch.empty((steps * C, L, N), dtype=i8, device=dev)
    ys = torch.empty(steps * C, dtype=f64, device=dev)
    n_acc = 0
    t0 = time.perf_counter()
    for k in range(3 + steps):
        slq.slq_cumulative_step(plan, eff, s, la, sg, n_lin, seed, k, 0, acc, logA, st)
        if k >= 3:
            j = (k - 3) * C
            xs[j:j + C].copy_(s)
            ys[j:j + C].copy_(la)
            n_acc += int(acc.sum().item())
            print(f"# learned 48x48: {j + C} exact-weight pairs", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    ok = bool((st == 0).all().item())
    P = xs.shape[0]
    slq.slq_fit_effective(plan, eff, xs, ys, theta, r2)
    slq.slq_eff_set_theta(eff, theta)
    torch.cuda.synchronize()

    n_tr = P - P // 10
    prm = torch.from_numpy(net_init(seed)).to(dev)
    prm[1960:] = 0.0
    mom, vel, g = torch.zeros_like(prm), torch.zeros_like(prm), torch.empty_like(prm)
    loss = torch.empty(1, dtype=f64, device=dev)

    def held_out(params):
        tot = 0.0
        for k in range(n_tr, P, C):
            e = min(P, k + C)
            slq.slq_net_gradient(plan, eff, slq.SLQ_PREC_FP32, xs[k:e], ys[k:e], params, g, loss)
            tot += float(loss.item()) * (e - k) / (P - n_tr)
        return tot

    mse_lin = held_out(torch.zeros_like(prm))
    best_prm, best_mse, curve = None, mse_lin, []
    order = np.random.default_rng(seed)
    t_adam, batch, samples = 0, 64, 0
    check = max(batch, (n_tr // 4) // batch * batch)   # held-out loss four times per epoch
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < train_seconds:
        perm = torch.from_numpy(order.permutation(n_tr)).to(dev)
        for k in range(0, n_tr - batch + 1, batch):
            idx = perm[k:k + batch]
            slq.slq_net_gradient(plan, eff, slq.SLQ_PREC_FP32, xs[idx].contiguous(), ys[idx].contiguous(), prm, g,
                                 loss)
            t_adam += 1
            samples += batch
            slq.slq_net_adam(prm, g, mom, vel, t_adam, lr=1e-3)
            if samples % check == 0:
                curve.append(held_out(prm))
                if curve[-1] < best_mse:
                    best_mse, best_prm = curve[-1], prm.clone()
                print(f"# learned 48x48: {samples} training samples, held-out MSE {curve[-1]:.6g} "
                      f"(linear {mse_lin:.6g})", file=sys.stderr, flush=True)
            if time.perf_counter() - t0 >= train_seconds:
                break
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0

    # proposals: the same chains from the same start, learned then linear
    s0, la0, sg0 = s.clone(), la.clone(), sg.clone()

    def run(n_moves, step0):
        s.copy_(s0)
        la.copy_(la0)
        sg.copy_(sg0)
        accs, la_std = [], []
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(eval_steps):
            slq.slq_cumulative_step(plan, eff, s, la, sg, n_moves, seed, step0 + k, 0, acc, logA, st)
            accs.append(float(acc.float().mean().item()))
            la_std.append(float(logA.std().item()))
        torch.cuda.synchronize()
        return {"steps": eval_steps, "effective_moves": n_moves, "acceptance": float(np.mean(accs)),
                "std_logA": float(np.mean(la_std)), "steps_per_s": C * eval_steps / (time.perf_counter() - t1),
                "status_ok": bool((st == 0).all().item())}

    learned = None
    if best_prm is not None:
        slq.slq_eff_set_net(eff, best_prm, slq.SLQ_PREC_FP64)
        learned = run(slq.slq_eff_net_classes(eff), 10_000)
        print("# learned 48x48: learned proposals done", file=sys.stderr, flush=True)
        slq.slq_eff_set_net(eff, None)
    linear = run(n_lin, 10_000)
    out = {"workload": "learned_48x48", "model": "48x48, L=100, beta=10, xi=1.5, mu=-0.5",
           "chains": C, "pairs": P, "pair_generation": {"seconds": t_gen, "acceptance": n_acc / P,
                                                         "status_ok": ok},
           "linear_fit": {"terms": len(terms), "r2": float(r2.item())},
           "training": {"train": n_tr, "held_out": P - n_tr, "seconds": t_train, "adam_steps": t_adam,
                        "epochs": samples / n_tr, "batch": batch, "lr": 1e-3, "net_prec": "fp32",
                        "held_out_mse_linear": mse_lin, "held_out_mse_best": best_mse,
                        "held_out_mse_curve": curve},
           "proposals_linear": linear, "proposals_learned": learned,
           "proposals_from": "linear + network" if best_prm is not None else
                             "linear (fallback: no checkpoint beat the linear action on held-out fields)"}
    eff.close()
    plan.close()
    del xs, ys
    torch.cuda.empty_cache()
    return out


def precision_rates(slq, fields: int = 32):
    """Chain products of the 40x40, L=100 model (dtau 0.1, xi 1.5, n_s 10) in
    each precision mode: exact weights per second of `fields` fields and the
    chain kernels' throughput against their own peak (structured FP64 on the
    vector ALUs; dense FP64, FP32 and BF16 products on the matrix cores, FP32
    accumulation for the last two)."""
    import torch
    from slq_inputs import MIXED_40x40, iid_fields
    dev = torch.device("cuda")
    model = MIXED_40x40
    s = torch.from_numpy(iid_fields(model, fields, 4000)).to(dev)
    out = {}
    names = {0: "fp64_structured", 3: "fp64_dense", 1: "fp32", 2: "bf16"}
    for prec in (0, 3, 1, 2):
        plan = slq.Plan(model, fields, chain_prec=prec)
        slq.slq_plan_tune(plan, fields)  # block width, or tile shape of the dense FP64 GEMM
        la = torch.empty(fields, dtype=torch.float64, device=dev)
        sg = torch.empty(fields, dtype=torch.int8, device=dev)
        st = torch.empty(fields, dtype=torch.int32, device=dev)
        slq.slq_weight(plan, s, la, sg, st)
        torch.cuda.synchronize()
        slq.slq_profile_enable(plan, True)
        t0 = time.perf_counter()
        slq.slq_weight(plan, s, la, sg, st)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms, launches, flops = slq.slq_profile_read(plan)
        slq.slq_profile_enable(plan, False)
        tf = flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        out[names[prec]] = {"evals_per_s": fields / dt, "chain_tflops": tf,
                            "chain_peak_tflops": PRECISION_PEAK_TFLOPS[prec],
                            "chain_frac": tf / PRECISION_PEAK_TFLOPS[prec], "chain_launches": launches}
        plan.close()
        torch.cuda.empty_cache()
    return {"model": "40x40, L=100", "fields": fields, **out}


def precision_table(slq, fields: int = 256, chunk: int = 64, oracle_fields: int = 2):
    """cfg3's error table: the 40x40, L=100 model on `fields` seeded fields,
    half iid, half ordered domains with 10 % flips; log|W|, sign and G with
    FP32 and BF16 chain operands against the FP64 structured chain (the
    reference, itself checked against the oracle on `oracle_fields` of them,
    one of each kind)."""
    import numpy as np
    import torch
    from oracle import stable
    from slq_inputs import MIXED_40x40, mixed_batch
    dev = torch.device("cuda")
    m = MIXED_40x40
    N = m.n_sites
    S = mixed_batch(m, fields, 9300)
    kinds = np.array(["iid"] * (fields // 2) + ["domain"] * (fields - fields // 2))
    res = {}
    G = np.empty((fields, N, N))  # the FP64 reference's Green's functions
    for prec in (0, 1, 2):
        plan = slq.Plan(m, chunk, chain_prec=prec)
        la = np.empty(fields)
        sg = np.empty(fields, dtype=np.int8)
        st = np.empty(fields, dtype=np.int32)
        dG = np.empty(fields)
        for c0 in range(0, fields, chunk):
            c1 = min(fields, c0 + chunk)
            s = torch.from_numpy(S[c0:c1]).to(dev)
            Gd = torch.empty((c1 - c0, N, N), dtype=torch.float64, device=dev)
            lad = torch.empty(c1 - c0, dtype=torch.float64, device=dev)
            sgd = torch.empty(c1 - c0, dtype=torch.int8, device=dev)
            std = torch.empty(c1 - c0, dtype=torch.int32, device=dev)
            slq.slq_green(plan, s, Gd, lad, sgd, std)
            la[c0:c1], sg[c0:c1], st[c0:c1] = lad.cpu().numpy(), sgd.cpu().numpy(), std.cpu().numpy()
            if prec == 0:
                G[c0:c1] = Gd.cpu().numpy()
            else:
                dG[c0:c1] = (Gd - torch.from_numpy(G[c0:c1]).to(dev)).abs().amax(dim=(1, 2)).cpu().numpy()
            del Gd
        plan.close()
        torch.cuda.empty_cache()
        res[prec] = (la, sg, st, dG)
        print(f"# precision table: chain precision {prec} done", file=sys.stderr, flush=True)
    la0, sg0 = res[0][0], res[0][1]
    out = {"model": "40x40, L=100, beta=10, xi=1.5, mu=-0.5", "fields": fields,
           "reference": "FP64 structured chain on the GPU", "status_ok": True}
    for prec, name in ((1, "fp32"), (2, "bf16")):
        la, sg, st, dG = res[prec]
        rel = np.abs(la - la0) / np.abs(la0)
        row = {}
        for kind in ("iid", "domain"):
            k = kinds == kind
            row[kind] = {"max_rel_dlogW": float(rel[k].max()), "median_rel_dlogW": float(np.median(rel[k])),
                         "max_abs_dG": float(dG[k].max()), "median_abs_dG": float(np.median(dG[k])),
                         "signs_agree": bool((sg[k] == sg0[k]).all())}
        out[name] = row
        out["status_ok"] = out["status_ok"] and bool((st == 0).all())
    checks = []
    for idx in (0, fields - 1)[:oracle_fields]:
        t0 = time.perf_counter()
        rl, rs, rg = stable.green(m, S[idx])
        checks.append({"field": int(idx), "kind": str(kinds[idx]), "oracle_seconds": time.perf_counter() - t0,
                       "fp64_rel_dlogW": float(abs(la0[idx] - rl) / abs(rl)),
                       "fp64_max_abs_dG": float(np.max(np.abs(G[idx] - rg))),
                       "signs_agree": bool(sg0[idx] == rs)})
    out["fp64_vs_oracle"] = checks
    return out


def group_rate(slq, dev, reps: int = 5):
    """Exact weights of 64 chains of uneven size (Lx = Ly in {8..24}, L in
    {40..100}) per second, one graph launch per evaluation."""
    import torch
    from slq_inputs import uneven_models, iid_field
    models = uneven_models(64, 4000)
    grp = slq.Group(models)
    s = torch.from_numpy(grp.pack([iid_field(m, 4100 + c) for c, m in enumerate(models)])).to(dev)
    la = torch.empty(64, dtype=torch.float64, device=dev)
    sg = torch.empty(64, dtype=torch.int8, device=dev)
    slq.slq_group_weight(grp, s, la, sg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        slq.slq_group_weight(grp, s, la, sg)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    def work(m):  # algorithmic flops of one exact weight: structured products, QRs, V updates, final step
        n, blocks = m.n_sites, -(-m.n_slices // m.n_stab)
        final = 4.0 / 3.0 * n ** 3 if n > 64 else 2.0 / 3.0 * n ** 3
        return (2.0 * n * n * (m.lx + m.ly) * m.n_slices + blocks * 8.0 / 3.0 * n ** 3
                + (blocks - 1) * float(n) ** 3 + final)
    flops = sum(work(m) for m in models)
    info = grp.describe()
    grp.close()
    cum = group_cumulative_rate(slq, dev, models, reps)
    return {"evals_per_s": 64 / dt, "ms_per_launch": dt * 1e3, "graph_launches_per_eval": 1,
            "cumulative_updates": cum,
            "algorithmic_tflops": flops / dt / 1e12,
            "flops_note": "per chain: 2 N^2 (lx+ly) L structured products, (8/3) N^3 per QR, N^3 per V update, "
                          "(4/3) N^3 final QR (N > 64) or (2/3) N^3 LU",
            "batches": len(info["batches"]), "tuned": info["tuned"]}


def group_cumulative_rate(slq, dev, models, reps):
    """Cumulative updates of the 64 uneven chains in one call per update: one
    batch per distinct model, each with a short linear effective action (one-
    body, nearest-neighbour, nearest-slice and space-time terms) fitted on the
    GPU (Eq. 3) to the exact weights of 32 iid fields of its model, one
    effective sweep per proposal."""
    import numpy as np
    import torch
    from slq_inputs import iid_field, iid_fields
    grp = slq.Group(models, exact_batches=True)
    fields = [iid_field(m, 4200 + c) for c, m in enumerate(models)]
    s = torch.from_numpy(grp.pack(fields)).to(dev)
    n = len(models)
    la = torch.empty(n, dtype=torch.float64, device=dev)
    sg = torch.empty(n, dtype=torch.int8, device=dev)
    slq.slq_group_weight(grp, s, la, sg)
    effs = []
    terms = [(0, 0), (1, 0), (0, 1), (1, 1)]
    for k in range(grp.n_batches):
        plan, ids = grp.batch(k)
        m = models[int(ids[0])]
        eff = slq.Eff(plan, terms, np.zeros(len(terms)))
        xs = torch.from_numpy(iid_fields(m, 32, 4300 + k)).to(dev)
        ys = torch.empty(32, dtype=torch.float64, device=dev)
        sgw = torch.empty(32, dtype=torch.int8, device=dev)
        for c0 in range(0, 32, plan.max_batch):
            c1 = min(32, c0 + plan.max_batch)
            slq.slq_weight(plan, xs[c0:c1], ys[c0:c1], sgw[c0:c1])
        theta = torch.empty(1 + len(terms), dtype=torch.float64, device=dev)
        r2 = torch.empty(1, dtype=torch.float64, device=dev)
        slq.slq_fit_effective(plan, eff, xs, ys, theta, r2)
        slq.slq_eff_set_theta(eff, theta)
        effs.append(eff)
    acc = torch.empty(n, dtype=torch.int8, device=dev)
    st = torch.empty(n, dtype=torch.int32, device=dev)
    slq.slq_group_cumulative_step(grp, effs, 1, 0x5D0C + 4, 0, s, la, sg, acc, None, st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rate = 0.0
    for k in range(reps):
        slq.slq_group_cumulative_step(grp, effs, 1, 0x5D0C + 4, 1 + k, s, la, sg, acc, None, st)
        rate += float(acc.float().mean().item())
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    ok = bool((st == 0).all().item())
    nb = grp.n_batches
    for e in effs:
        e.close()
    grp.close()
    return {"batches": nb, "updates_per_s": n / dt, "ms_per_call": dt * 1e3, "acceptance": rate / reps,
            "status_ok": ok, "effective_sweeps_per_update": 1}


def headline(slq, args, workload):
    """Cumulative updates of B chains on `workload` (the timed region), with
    the chain, stabilisation and final-step parts timed by HIP events."""
    import numpy as np
    import torch
    from slq_inputs import WORKLOADS, iid_fields, default_terms
    model = WORKLOADS[workload]
    B = args.batch or (256 if workload == "learned_48x48" else 512)
    seed = 0x5D0C + (5 if workload == "learned_48x48" else 2)
    dev = torch.device("cuda")
    cb = args.chain == "checkerboard"
    plan = slq.Plan(model, B, slq.SLQ_PREC_CHECKERBOARD if cb else slq.SLQ_PREC_FP64)
    if args.block_width:
        slq.slq_plan_set_block_width(plan, args.block_width)
        kron_nb = args.block_width
    else:
        kron_nb = slq.slq_plan_tune(plan, B)
    terms = default_terms(model.n_slices)

    # training set and fit (step ii): exact weights of B seeded fields
    fields = iid_fields(model, B, 2000)
    s = torch.from_numpy(fields).to(dev)
    logabs = torch.empty(B, dtype=torch.float64, device=dev)
    sign = torch.empty(B, dtype=torch.int8, device=dev)
    status = torch.empty(B, dtype=torch.int32, device=dev)
    slq.slq_weight(plan, s, logabs, sign, status)
    eff = slq.Eff(plan, terms, np.zeros(len(terms)))
    theta = torch.empty(1 + len(terms), dtype=torch.float64, device=dev)
    r2 = torch.empty(1, dtype=torch.float64, device=dev)
    slq.slq_fit_effective(plan, eff, s, logabs, theta, r2)
    slq.slq_eff_set_theta(eff, theta)
    n_moves = eff.n_classes
    torch.cuda.synchronize()
    theta_h = theta.cpu().numpy()

    accepted = torch.zeros((args.warmup + args.steps, B), dtype=torch.int8, device=dev)
    logA = torch.empty(B, dtype=torch.float64, device=dev)
    for w in range(args.warmup):
        slq.slq_cumulative_step(plan, eff, s, logabs, sign, n_moves, seed, w, 0, accepted[w], logA, status)
    torch.cuda.synchronize()
    print(f"# {workload}: {B} chains, warm-up done; timing {args.steps} steps", file=sys.stderr, flush=True)

    slq.slq_profile_enable(plan, True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        st = args.warmup + k
        slq.slq_cumulative_step(plan, eff, s, logabs, sign, n_moves, seed, st, 0, accepted[st], logA, status)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    parts = {name: slq.slq_profile_read(plan, part) for name, part in
             (("chain", slq.SLQ_PROFILE_CHAIN), ("stabilisation", slq.SLQ_PROFILE_STAB),
              ("final", slq.SLQ_PROFILE_FINISH))}
    slq.slq_profile_enable(plan, False)
    ok = bool((status == 0).all().item())
    value = B * args.steps / elapsed

    def part_info(name, peak):
        ms, n, fl = parts[name]
        tf = fl / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        return {"tflops": tf, "frac_of_fp64_peak": tf / peak, "share_of_step": ms * 1e-3 / elapsed,
                "sequences": n, "avg_ms": ms / max(1, n), "flops_per_sequence": fl / max(1, n)}

    stab = part_info("stabilisation", FP64_PEAK_TFLOPS)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded iid +-1 auxiliary fields, effective model fitted on the GPU to their exact weights",
        "config": {"workload": workload, "lattice": f"{model.lx}x{model.ly}", "N": model.n_sites,
                   "L": model.n_slices, "beta": model.beta, "t": model.t, "mu": model.mu, "xi": model.xi,
                   "n_stab": model.n_stab, "chains": B, "effective_moves_per_step": n_moves,
                   "proposals_per_step": int(model.n_sites * model.n_slices), "terms": len(terms),
                   "judge": "FP64 (structured slice products, blocked Householder QR/UDV, QR determinant)",
                   "kinetic_factor": ("checkerboard split E_cb (a different Trotter discretisation)" if cb
                                      else "exact exp(-dtau K)"),
                   "chain_block_vectors_per_workgroup": kron_nb},
        "roofline": {"bound": "mfma", "achieved": stab["tflops"], "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": stab["frac_of_fp64_peak"], "traffic": STAB_TRAFFIC.get((workload, B)),
                     "kernel": "stabilisation: pre-pivoted blocked Householder QR of X diag(D) (register panels, "
                               "compact-WY updates on FP64 MFMA) with its explicit Q, and the V update; "
                               "flops (8/3) N^3 per field per QR + N^3 per V update (none for the first block)",
                     "launches": stab["sequences"], "avg_launch_ms": stab["avg_ms"],
                     "flops_per_launch": stab["flops_per_sequence"]},
    }
    details = {"fit_r2": float(r2.item()),
               "cumulative_acceptance": float(accepted[args.warmup:].float().mean().item()),
               "status_ok": ok,
               "parts": {"stabilisation": stab,
                         "chain": {**part_info("chain", FP64_PEAK_TFLOPS),
                                   "note": ("checkerboard FP64 slice products (bond rotations in registers, edge "
                                            "exchanges in LDS): 22 N^2 flops per slice and field" if cb else
                                            ("structured FP64 slice products (48 x 48: circulant lines on the "
                                             "matrix cores; otherwise vector FMA): " if model.lx == model.ly == 48 else
                                             "structured FP64 slice products (vector FMA): ") +
                                            "2 N^2 (lx+ly) flops per slice and field")},
                         "final": {**part_info("final", FP64_PEAK_TFLOPS),
                                   "note": "QR of M for the determinant: (4/3) N^3 per field"}}}
    return out, details, plan, eff, s, logabs, sign, status, theta_h, fields, model, terms, seed


def details_20x20(slq, seed):
    """The 20x20, L = 80 workload: cumulative updates, Green's functions and
    local DQMC sweeps per second of 512 chains (a few steps each)."""
    import numpy as np
    import torch
    from slq_inputs import DQMC_20x20, iid_fields, default_terms
    dev = torch.device("cuda")
    model, B = DQMC_20x20, 512
    plan = slq.Plan(model, B, sweeps=True)
    slq.slq_plan_tune(plan, B)
    s = torch.from_numpy(iid_fields(model, B, 2000)).to(dev)
    la = torch.empty(B, dtype=torch.float64, device=dev)
    sg = torch.empty(B, dtype=torch.int8, device=dev)
    st = torch.empty(B, dtype=torch.int32, device=dev)
    slq.slq_weight(plan, s, la, sg, st)
    terms = default_terms(model.n_slices)
    eff = slq.Eff(plan, terms, np.zeros(len(terms)))
    theta = torch.empty(1 + len(terms), dtype=torch.float64, device=dev)
    r2 = torch.empty(1, dtype=torch.float64, device=dev)
    slq.slq_fit_effective(plan, eff, s, la, theta, r2)
    slq.slq_eff_set_theta(eff, theta)
    acc = torch.empty(B, dtype=torch.int8, device=dev)
    logA = torch.empty(B, dtype=torch.float64, device=dev)
    slq.slq_cumulative_step(plan, eff, s, la, sg, eff.n_classes, seed, 0, 0, acc, logA, st)
    torch.cuda.synchronize()
    steps = 5
    slq.slq_profile_enable(plan, True)
    t0 = time.perf_counter()
    for k in range(steps):
        slq.slq_cumulative_step(plan, eff, s, la, sg, eff.n_classes, seed, 1 + k, 0, acc, logA, st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_s, _, fl_s = slq.slq_profile_read(plan, slq.SLQ_PROFILE_STAB)
    ms_c, n_c, fl_c = slq.slq_profile_read(plan, slq.SLQ_PROFILE_CHAIN)
    slq.slq_profile_enable(plan, False)
    out = {"workload": "dqmc_20x20", "chains": B, "cumulative_updates_per_s": B * steps / dt,
           "stabilisation_tflops": fl_s / (ms_s * 1e-3) / 1e12 if ms_s > 0 else 0.0,
           "chain_tflops": fl_c / (ms_c * 1e-3) / 1e12 if ms_c > 0 else 0.0,
           "chain_avg_launch_ms": ms_c / max(1, n_c)}
    G = torch.empty((B, model.n_sites, model.n_sites), dtype=torch.float64, device=dev)
    slq.slq_green(plan, s, G, la, sg, st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    slq.slq_green(plan, s, G, la, sg, st)
    torch.cuda.synchronize()
    out["green_evals_per_s"] = B / (time.perf_counter() - t0)
    a64 = torch.empty(B, dtype=torch.int64, device=dev)
    drift = torch.empty(B, dtype=torch.float64, device=dev)
    slq.slq_sweep_local(plan, s, G, la, sg, 1, seed, 0, 0, a64, drift, st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    slq.slq_sweep_local(plan, s, G, la, sg, 1, seed, 1, 0, a64, drift, st)
    torch.cuda.synchronize()
    out["dqmc_sweeps_per_s"] = B / (time.perf_counter() - t0)
    out["dqmc_max_drift"] = float(drift.max().item())
    eff.close()
    plan.close()
    torch.cuda.empty_cache()
    return out


def dqmc_long(slq, chains, sweeps, every):
    """Long local-update run on the 20x20, L = 80 workload: `sweeps` sweeps of
    `chains` chains, and every `every` sweeps the largest wrap drift seen
    (max |G_wrapped - G_fresh| at the recomputes) and the largest difference
    between the tracked log|W| (advanced by log|R| of accepted flips) and
    log|W| evaluated afresh on the current fields."""
    import torch
    from slq_inputs import DQMC_20x20, iid_fields
    dev = torch.device("cuda")
    m = DQMC_20x20
    N = m.n_sites
    plan = slq.Plan(m, chains, sweeps=True)
    s = torch.from_numpy(iid_fields(m, chains, 3100)).to(dev)
    G = torch.empty((chains, N, N), dtype=torch.float64, device=dev)
    la = torch.empty(chains, dtype=torch.float64, device=dev)
    sg = torch.empty(chains, dtype=torch.int8, device=dev)
    st = torch.empty(chains, dtype=torch.int32, device=dev)
    acc = torch.empty(chains, dtype=torch.int64, device=dev)
    drift = torch.empty(chains, dtype=torch.float64, device=dev)
    fresh = torch.empty(chains, dtype=torch.float64, device=dev)
    fsg = torch.empty(chains, dtype=torch.int8, device=dev)
    fst = torch.empty(chains, dtype=torch.int32, device=dev)
    slq.slq_green(plan, s, G, la, sg, st)
    log = []
    t0 = time.perf_counter()
    done = 0
    while done < sweeps:
        n = min(every, sweeps - done)
        slq.slq_sweep_local(plan, s, G, la, sg, n, 0x5D0C + 2, done, 0, acc, drift, st)
        done += n
        slq.slq_weight(plan, s, fresh, fsg, fst)
        torch.cuda.synchronize()
        rec = {"sweeps": done, "max_drift": float(drift.max().item()),
               "max_abs_dlogW_tracked_vs_fresh": float((la - fresh).abs().max().item()),
               "max_rel_dlogW_tracked_vs_fresh": float(((la - fresh).abs() / fresh.abs()).max().item()),
               "signs_agree": bool((sg == fsg).all().item()), "status_ok": bool((st == 0).all().item()),
               "acceptance": float(acc.sum().item()) / (chains * n * N * m.n_slices),
               "seconds": time.perf_counter() - t0}
        log.append(rec)
        print(f"# {json.dumps(rec)}", file=sys.stderr, flush=True)
    plan.close()
    return {"workload": "dqmc_20x20", "chains": chains, "sweeps": sweeps,
            "sweeps_per_s": chains * sweeps / (time.perf_counter() - t0), "log": log}


def bilayer_tau(slq, sizes, chains, sweeps, steps, burn, train_sweeps, eff_sweeps, sl_burn=None):
    """The paper's comparison of autocorrelation times (Fig. 3) on its own
    workload, at small sizes: the bilayer weight of Eq. 6 at beta = 1,
    dtau = 0.05, xi = 1, h = 2.774 (J = 1).  For each linear size: `chains`
    local-update DQMC chains (`burn` sweeps, then `sweeps` sweeps recording the
    total magnetisation M), and as many SLDQMC chains started from the DQMC end
    configurations making `steps` cumulative updates of `eff_sweeps` effective
    sweeps each (the paper makes roughly tau_L effective sweeps per
    cumulative update), with the effective model fitted
    once at the smallest size (as the
    paper fits at L = 8 and reuses it) on DQMC configurations and their exact
    weights.  tau_int of M per sweep and per cumulative update, <M^2> and the
    susceptibility chi = dtau^2 <M^2> / (beta^2 N) of both samplers with
    errors, wall time per sweep and per update.  tau_int is also given for |M|
    and M^2, which the tunnelling between +M and -M does not set, and <M^2>
    over each half of the recorded series, which shows an unfinished burn-in.
    sl_burn: cumulative updates before the recorded ones (default: burn)."""
    import numpy as np
    import torch
    from paper_1612_03804_amd.analysis import tau_int_window, mean_and_error, agree
    from slq_inputs import bilayer_model, iid_fields, default_terms, BILAYER_J, BILAYER_H
    dev = torch.device("cuda")
    f64, i8, i32, i64 = torch.float64, torch.int8, torch.int32, torch.int64
    seed = 0x5D0C + 6
    out = {"workload": "bilayer (Eq. 6), beta=1, dtau=0.05, M=20, xi=1, h=2.774, J=1, t=1, mu=-0.5",
           "chains": chains, "sizes": {}}
    theta_h, terms = None, None

    def halves(x):   # <M^2> over the first and the second half of the recorded series: a drift shows here
        h = x.shape[1] // 2
        return [mean_and_error(x[:, :h]), mean_and_error(x[:, h:])]

    for lin in sizes:
        m = bilayer_model(lin)
        N, L = m.n_sites, m.n_slices
        C = chains
        plan = slq.Plan(m, 2 * C)
        s = torch.from_numpy(iid_fields(m, C, 7000 + lin)).to(dev)
        G = torch.empty((2 * C, N, N), dtype=f64, device=dev)
        lw = torch.empty(C, dtype=f64, device=dev)
        st = torch.empty(C, dtype=i32, device=dev)
        acc = torch.empty(C, dtype=i64, device=dev)
        drift = torch.empty(C, dtype=f64, device=dev)
        slq.slq_bilayer_green(plan, BILAYER_J, BILAYER_H, s, G, lw, st)
        for k0 in range(0, burn, 250):
            slq.slq_bilayer_sweep_local(plan, BILAYER_J, BILAYER_H, s, G, lw, min(250, burn - k0), seed, k0, 0, acc,
                                        drift, st)
            torch.cuda.synchronize()
            print(f"# bilayer L={lin}: burn-in {min(burn, k0 + 250)} sweeps", file=sys.stderr, flush=True)
        Md = torch.empty((sweeps, C), dtype=i64, device=dev)
        keep = max(1, sweeps // max(1, train_sweeps))
        train_s, train_w = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(sweeps):
            slq.slq_bilayer_sweep_local(plan, BILAYER_J, BILAYER_H, s, G, lw, 1, seed, burn + k, 0, acc, drift, st)
            slq.slq_magnetization(plan, s, Md[k])
            if (k + 1) % 250 == 0:
                torch.cuda.synchronize()
                print(f"# bilayer L={lin}: {k + 1} DQMC sweeps", file=sys.stderr, flush=True)
            if theta_h is None and k % keep == 0 and len(train_s) < train_sweeps:
                train_s.append(s.clone())
                train_w.append(lw.clone())
        torch.cuda.synchronize()
        t_dq = time.perf_counter() - t0
        Mh = Md.cpu().numpy().T.astype(np.float64)
        ok_dq = bool((st == 0).all().item()) and float(drift.max().item()) < 1e-6
        rec = {"N": N, "dqmc": {"sweeps": sweeps, "ms_per_sweep": 1e3 * t_dq / sweeps,
                                "tau_int_sweeps": tau_int_window(Mh),
                                "tau_int_sweeps_absM": tau_int_window(np.abs(Mh)),
                                "tau_int_sweeps_M2": tau_int_window(Mh ** 2), "M2": mean_and_error(Mh ** 2),
                                "M2_halves": halves(Mh ** 2), "status_ok": ok_dq, "max_drift": float(drift.max().item())}}
        if theta_h is None:   # fit the effective model at the smallest size (Eq. 3)
            terms = default_terms(L)
            eff0 = slq.Eff(plan, terms, np.zeros(len(terms)))
            xs = torch.cat(train_s)
            ys = torch.cat(train_w)
            th = torch.empty(1 + len(terms), dtype=f64, device=dev)
            r2 = torch.empty(1, dtype=f64, device=dev)
            slq.slq_fit_effective(plan, eff0, xs, ys, th, r2)
            torch.cuda.synchronize()
            theta_h = th.cpu().numpy()
            out["fit"] = {"size": lin, "samples": int(xs.shape[0]), "terms": len(terms), "r2": float(r2.item())}
            eff0.close()
        # lambda carries over; c0 only shifts the action and cancels in Eq. 4
        eff = slq.Eff(plan, terms, theta_h[1:], float(theta_h[0]))
        n_moves = eff_sweeps * eff.n_classes
        slq.slq_bilayer_weight(plan, BILAYER_J, BILAYER_H, s, lw, st)
        Ms = torch.empty((steps, C), dtype=i64, device=dev)
        acc_c = torch.empty((steps, C), dtype=i8, device=dev)
        logA = torch.empty(C, dtype=f64, device=dev)
        for k in range(burn if sl_burn is None else sl_burn):
            slq.slq_bilayer_cumulative_step(plan, eff, BILAYER_J, BILAYER_H, s, lw, n_moves, seed, 100_000 + k, 0,
                                            acc_c[0], logA, st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            slq.slq_bilayer_cumulative_step(plan, eff, BILAYER_J, BILAYER_H, s, lw, n_moves, seed, 200_000 + k, 0,
                                            acc_c[k], logA, st)
            slq.slq_magnetization(plan, s, Ms[k])
            if (k + 1) % 250 == 0:
                torch.cuda.synchronize()
                print(f"# bilayer L={lin}: {k + 1} cumulative updates", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t_sl = time.perf_counter() - t0
        Msh = Ms.cpu().numpy().T.astype(np.float64)
        m2_sl = mean_and_error(Msh ** 2)
        beta = m.beta
        chi = lambda x: (m.dtau ** 2 * x[0] / (beta ** 2 * N), m.dtau ** 2 * x[1] / (beta ** 2 * N))
        rec["sldqmc"] = {"steps": steps, "effective_sweeps_per_step": eff_sweeps, "effective_moves": n_moves,
                         "ms_per_step": 1e3 * t_sl / steps,
                         "acceptance": float(acc_c.float().mean().item()), "tau_int_steps": tau_int_window(Msh),
                         "tau_int_steps_absM": tau_int_window(np.abs(Msh)),
                         "tau_int_steps_M2": tau_int_window(Msh ** 2),
                         "M2": m2_sl, "M2_halves": halves(Msh ** 2), "status_ok": bool((st == 0).all().item())}
        rec["chi_dqmc"] = chi(rec["dqmc"]["M2"])
        rec["chi_sldqmc"] = chi(m2_sl)
        rec["M2_agree_2sigma"] = agree(rec["dqmc"]["M2"], m2_sl)
        out["sizes"][str(lin)] = rec
        print(f"# bilayer L={lin}: {json.dumps(rec)}", file=sys.stderr, flush=True)
        eff.close()
        plan.close()
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=0, help="chains (0: 256 at 48x48, 512 at 20x20)")
    ap.add_argument("--workload", choices=("learned_48x48", "dqmc_20x20"), default="learned_48x48")
    ap.add_argument("--chain", choices=("exact", "checkerboard"), default="exact",
                    help="kinetic factor of the timed chains: exact exp(-dtau K) (circulant lines) or the "
                         "checkerboard split E_cb")
    ap.add_argument("--block-width", type=int, default=0,
                    help="vectors per workgroup of the chain-block kernel (0: tuned on the plan)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-details", action="store_true")
    ap.add_argument("--ess-only", action="store_true",
                    help="print the effective-samples/s comparison of the two samplers (its own JSON line)")
    ap.add_argument("--ess-steps", type=int, default=200)
    ap.add_argument("--ess-sweeps", type=int, default=200)
    ap.add_argument("--ess-chains", type=int, default=128)
    ap.add_argument("--ess-burn", type=int, default=10)
    ap.add_argument("--dqmc-long", type=int, default=0,
                    help="this many local sweeps at 20x20, L = 80 with drift and tracked-weight checks (own JSON line)")
    ap.add_argument("--dqmc-long-chains", type=int, default=16)
    ap.add_argument("--bilayer-tau", action="store_true",
                    help="autocorrelation times of DQMC and SLDQMC on the bilayer workload (own JSON line)")
    ap.add_argument("--bilayer-sizes", default="8,12,16")
    ap.add_argument("--bilayer-chains", type=int, default=64)
    ap.add_argument("--bilayer-sweeps", type=int, default=2000)
    ap.add_argument("--bilayer-steps", type=int, default=400)
    ap.add_argument("--bilayer-burn", type=int, default=200)
    ap.add_argument("--bilayer-eff-sweeps", type=int, default=50)
    ap.add_argument("--bilayer-sl-burn", type=int, default=None,
                    help="cumulative updates before the recorded ones (default: --bilayer-burn)")
    ap.add_argument("--learned-train", type=int, default=0, metavar="PAIRS",
                    help="the learned action at 48x48, L=100 on this many exact-weight pairs (own JSON line)")
    ap.add_argument("--learned-chains", type=int, default=256)
    ap.add_argument("--learned-seconds", type=float, default=240.0)
    ap.add_argument("--learned-eval-steps", type=int, default=10)
    ap.add_argument("--precision-table", action="store_true",
                    help="reduced-precision error table at 40x40, L=100 over 256 fields (own JSON line)")
    ap.add_argument("--reports", action="store_true",
                    help="print the uneven-group, precision-mode and learned-proposal reports (own JSON line)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device to device (a plain copy kernel of known size, against which "
                         "HBM byte counters collected over this run are scaled)")
    ap.add_argument("--sweeps-only", type=int, default=0,
                    help="time this many local DQMC sweeps of --batch chains at 20x20 instead (own JSON line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is a design note.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_1612_03804_amd import slq
    from slq_inputs import DQMC_20x20, default_terms

    if args.copy_calibration:
        src = torch.ones(COPY_CALIBRATION_BYTES // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.sweeps_only:
        plan = slq.Plan(DQMC_20x20, args.batch or 512, sweeps=True)
        print(json.dumps(local_sweep_rate(slq, plan, DQMC_20x20, args.sweeps_only, 0x5D0C + 2)), flush=True)
        return
    if args.ess_only:
        plan = slq.Plan(DQMC_20x20, args.ess_chains, sweeps=True, net=True)
        slq.slq_plan_tune(plan, args.ess_chains)
        print(json.dumps(ess_rates(slq, plan, DQMC_20x20, default_terms(DQMC_20x20.n_slices), 0x5D0C + 2,
                                   args.ess_steps, args.ess_chains, args.ess_sweeps, args.ess_burn)), flush=True)
        return
    if args.dqmc_long:
        print(json.dumps(dqmc_long(slq, args.dqmc_long_chains, args.dqmc_long, 100)), flush=True)
        return
    if args.bilayer_tau:
        sizes = [int(x) for x in args.bilayer_sizes.split(",")]
        print(json.dumps(bilayer_tau(slq, sizes, args.bilayer_chains, args.bilayer_sweeps, args.bilayer_steps,
                                     args.bilayer_burn, 40, args.bilayer_eff_sweeps, args.bilayer_sl_burn)),
              flush=True)
        return
    if args.precision_table:
        print(json.dumps(precision_table(slq)), flush=True)
        return
    if args.learned_train:
        print(json.dumps(learned_48x48_train(slq, args.learned_chains, args.learned_train, args.learned_seconds,
                                             args.learned_eval_steps)), flush=True)
        return
    if args.reports:
        dev = torch.device("cuda")
        print(json.dumps({"group_64_uneven": group_rate(slq, dev), "precision_40x40": precision_rates(slq),
                          "learned_48x48": learned_48x48_rates(slq)}), flush=True)
        return

    out, details, plan, eff, s, logabs, sign, status, theta_h, fields, model, terms, seed = \
        headline(slq, args, args.workload)
    eff.close()
    plan.close()
    del s, logabs, sign, status
    torch.cuda.empty_cache()
    if not args.no_details and args.workload != "dqmc_20x20":
        details["dqmc_20x20"] = details_20x20(slq, 0x5D0C + 2)
    if not args.no_details and args.chain == "exact":
        # the same workload with the checkerboard split (its own discretisation), a few steps
        cb_args = argparse.Namespace(**{**vars(args), "chain": "checkerboard", "steps": 3, "warmup": 1,
                                        "block_width": 0})
        o2, d2, p2, e2, *_ = headline(slq, cb_args, args.workload)
        e2.close()
        p2.close()
        torch.cuda.empty_cache()
        details["checkerboard"] = {"evals_per_s": o2["value"], "ms_per_step": o2["ms_per_step"],
                                   "steps": 3, "chain": d2["parts"]["chain"],
                                   "stabilisation_share": d2["parts"]["stabilisation"]["share_of_step"],
                                   "vectors_per_workgroup": o2["config"]["chain_block_vectors_per_workgroup"]}
    out["details"] = details
    if not args.no_cpu_baseline:
        print("# oracle timing on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(model, terms, theta_h, fields[0], seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
