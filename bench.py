#!/usr/bin/env python3
"""Benchmark of the self-learning DQMC hot path on one MI355X.

Workload: the 20x20 lattice (N = 400 sites), L = 80 slices (beta = 8,
dtau = 0.1), t = 1, mu = -0.5, xi = 1.5, QR stabilisation every 10 slices,
FP64 throughout.  A batch of B independent chains starts from seeded iid
+-1 fields; the linear effective action (default 1 + 2 + 40 + 4 = 47 terms)
is fitted on the GPU to their exact weights.

One timed step = one cumulative update (steps iii-iv of the method, Eq. 4) of
every chain: one sweep of colour-class effective moves, the exact weight of
the proposal (8 blocks of 10 slice products and 8 QR stabilisations, LU
log-det and sign) and the accept/reject.  Each step therefore makes exactly
B exact fermion-weight evaluations, and value = B * steps / seconds.

Also printed (same JSON line): the roofline of the chain-block kernel (the
structured slice products of a block of 10 slices, FP64 on the vector ALUs,
timed with HIP events on its stream over the timed region), the CPU oracle
timed on a bounded sample of the same workload, and untimed-for-value
details: acceptance, Green's-function evaluations/s, local DQMC sweeps/s,
uneven batches, the chain products of each precision mode at 40x40, the
48x48 workload's exact weights and cumulative updates (linear and learned
proposals), and the
effective samples per second of self-learning DQMC against local FP64 DQMC
with as many chains: with the linear effective action and FP64 judge, with
FP32 chain products in the judge (its error stated), and with proposals from
the trained network action (skip with --no-ess).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "exact fermion-weight evals/sec + effective indep. samples/sec vs FP64 DQMC"
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector (and matrix) peak
COPY_CALIBRATION_BYTES = 1 << 30
# HBM bytes per k_kron launch at batch 512, by vectors per workgroup, averaged
# over the 8 blocks of an evaluation (the first block starts from the identity
# and reads no X): rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, each scaled by
# what the same counter reads for the 1 GiB copy of --copy-calibration.
KRON_TRAFFIC_BATCH = 512
KRON_TRAFFIC = {8: 1.2676e9, 16: 1.2475e9}


def cpu_baseline(model, terms, theta, fields, logabs, signs, steps, seed):
    """The oracle's cumulative update on one chain, timed on the host cores."""
    import numpy as np
    from oracle import effective, stable
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    c0, lam = float(theta[0]), np.asarray(theta[1:], dtype=np.float64)
    classes = effective.colour_classes(model, terms)
    s = fields[0].copy()
    la, sg = float(logabs[0]), int(signs[0])
    n_moves = len(classes)
    effective.cumulative_step(model, terms, c0, lam, s.copy(), la, sg, 1, lambda x: stable.weight(model, x),
                              seed=seed, step=10 ** 6, classes=classes)      # warm-up (imports, BLAS threads)
    t0 = time.perf_counter()
    for k in range(steps):
        s, la, sg, _, _ = effective.cumulative_step(model, terms, c0, lam, s, la, sg, n_moves,
                                                    lambda x: stable.weight(model, x), seed=seed, step=k,
                                                    classes=classes)
    dt = time.perf_counter() - t0
    return {"value": steps / dt, "unit": "evals/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{steps} cumulative updates of one chain at 20x20, L=80 ({n_moves} effective moves "
                      f"and one exact weight each), {dt:.1f} s"}


def ess_rates(slq, plan, model, terms, seed, steps, n_dq, sweeps, burn):
    """Effective independent samples per second of the total magnetisation,
    following the self-learning procedure: (i) local DQMC sweeps on n_dq
    chains, timed, whose configurations and exact weights form the training
    set; (ii) the effective model fitted to them; (iii)+(iv) cumulative updates
    on all chains of the plan, started from the DQMC configurations, for a few
    numbers of effective moves per update."""
    import numpy as np
    import torch
    from paper_1612_03804_amd.analysis import tau_int_chains
    from slq_inputs import iid_fields
    dev = torch.device("cuda")
    B, L, N, n = plan.max_batch, model.n_slices, model.n_sites, n_dq
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
    train_s = torch.empty((sweeps, n, L, N), dtype=i8, device=dev)
    train_la = torch.empty((sweeps, n), dtype=f64, device=dev)
    Md = torch.empty((sweeps, n), dtype=i64, device=dev)
    acc_dq = torch.zeros(n, dtype=i64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(sweeps):
        slq.slq_sweep_local(plan, s_dq, G, la, sg, 1, seed, 1000 + k, 0, a64, drift, st)
        slq.slq_magnetization(plan, s_dq, Md[k])
        train_s[k].copy_(s_dq)
        train_la[k].copy_(la)
        acc_dq += a64
    torch.cuda.synchronize()
    t_dq = time.perf_counter() - t0
    tau_dq = tau_int_chains(Md.cpu().numpy().T)
    ess_dq = n * sweeps / (2 * tau_dq) / t_dq

    # (ii) fit on the DQMC configurations
    eff = slq.Eff(plan, terms, np.zeros(len(terms)))
    theta = torch.empty(1 + len(terms), dtype=f64, device=dev)
    r2 = torch.empty(1, dtype=f64, device=dev)
    slq.slq_fit_effective(plan, eff, train_s.view(-1, L, N), train_la.view(-1), theta, r2)
    slq.slq_eff_set_theta(eff, theta)

    # (iii)+(iv) cumulative updates from the DQMC end configurations
    start = s_dq.repeat((B + n - 1) // n, 1, 1)[:B].contiguous()

    def cumulative_run(pl, ef, n_moves):
        s = start.clone()
        logabs = torch.empty(B, dtype=f64, device=dev)
        sign = torch.empty(B, dtype=i8, device=dev)
        status = torch.empty(B, dtype=i32, device=dev)
        slq.slq_weight(pl, s, logabs, sign, status)
        acc = torch.empty((steps, B), dtype=i8, device=dev)
        logA = torch.empty((steps, B), dtype=f64, device=dev)
        M = torch.empty((steps, B), dtype=i64, device=dev)
        for k in range(burn):
            slq.slq_cumulative_step(pl, ef, s, logabs, sign, n_moves, seed, 10_000 + k, 0, acc[0], logA[0], status)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            slq.slq_cumulative_step(pl, ef, s, logabs, sign, n_moves, seed, 20_000 + k, 0, acc[k], logA[k], status)
            slq.slq_magnetization(pl, s, M[k])
        torch.cuda.synchronize()
        t_sl = time.perf_counter() - t0
        rate = float(acc.float().mean().item())
        la_h = logA.cpu().numpy()
        run = {"effective_moves": n_moves, "acceptance": rate, "logA_mean": float(la_h.mean()),
               "logA_std": float(la_h.std()), "steps_per_s": B * steps / t_sl}
        if rate > 0:   # a chain that never moves has no autocorrelation time
            tau_sl = tau_int_chains(M.cpu().numpy().T)
            run.update(tau_int_steps=tau_sl, ess_per_s=B * steps / (2 * tau_sl) / t_sl)
        else:
            run.update(tau_int_steps=None, ess_per_s=0.0)
        return run, s

    runs = [cumulative_run(plan, eff, n_moves)[0]
            for n_moves in (max(1, eff.n_classes // 4), eff.n_classes, 4 * eff.n_classes)]
    best = max(runs, key=lambda r: r["ess_per_s"])
    n_best = best["effective_moves"]

    # the same update with the chain products in FP32 (stabilisation, LU and
    # Eq. 4 in FP64); its judge's error is measured on the configurations it
    # sampled, against the FP64 weights of the same fields
    plan32 = slq.Plan(model, B, chain_prec=slq.SLQ_PREC_FP32)
    eff32 = slq.Eff(plan32, terms, np.zeros(len(terms)))
    slq.slq_eff_set_theta(eff32, theta)
    run32, s32 = cumulative_run(plan32, eff32, n_best)
    la64 = torch.empty(B, dtype=f64, device=dev)
    la32 = torch.empty(B, dtype=f64, device=dev)
    sg_w = torch.empty(B, dtype=i8, device=dev)
    st_w = torch.empty(B, dtype=i32, device=dev)
    slq.slq_weight(plan, s32, la64, sg_w, st_w)
    slq.slq_weight(plan32, s32, la32, sg_w, st_w)
    run32["max_abs_dlogW_vs_fp64"] = float((la32 - la64).abs().max().item())
    run32["max_rel_dlogW_vs_fp64"] = float(((la32 - la64).abs() / la64.abs().clamp(min=1.0)).max().item())
    eff32.close()
    plan32.close()

    # proposals from the learned action S_lin + S_net: the network (FP32
    # kernels, Adam) is trained on the residual of the linear fit over the same
    # DQMC configurations, 90 % for training and 10 % held out; its output layer
    # starts at zero, so training starts from the linear model.  The epoch with
    # the lowest held-out error is kept; if none beats the linear model alone,
    # the linear model is the fallback and proposes the updates
    from slq_inputs import net_init
    xs, ys = train_s.view(-1, L, N), train_la.view(-1)
    n_all = xs.shape[0]
    n_tr = n_all - n_all // 10
    prm = torch.from_numpy(net_init(seed)).to(dev)
    prm[1960:] = 0.0
    mom, vel, g = torch.zeros_like(prm), torch.zeros_like(prm), torch.empty_like(prm)
    loss = torch.empty(1, dtype=f64, device=dev)

    def held_out(params):
        tot = 0.0
        for k in range(n_tr, n_all, 256):
            e = min(n_all, k + 256)
            slq.slq_net_gradient(plan, eff, slq.SLQ_PREC_FP32, xs[k:e].contiguous(), ys[k:e].contiguous(), params,
                                 g, loss)
            tot += float(loss.item()) * (e - k) / (n_all - n_tr)
        return tot

    mse_lin = held_out(torch.zeros_like(prm))
    best_prm, best_mse, curve = None, mse_lin, []
    order = np.random.default_rng(seed)
    t_adam, batch, epochs = 0, 64, 6
    torch.cuda.synchronize()
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
        slq.slq_eff_set_net(eff, best_prm, slq.SLQ_PREC_FP32)
    run_net, _ = cumulative_run(plan, eff, n_best)
    run_net["training"] = {"samples": n_tr, "held_out": n_all - n_tr, "epochs": epochs, "adam_steps": t_adam,
                           "seconds": t_train, "held_out_mse_linear": mse_lin, "held_out_mse_by_epoch": curve,
                           "proposals_from": "linear + network" if best_prm is not None else
                           "linear (fallback: no epoch beat the linear model on held-out fields)"}
    slq.slq_eff_set_net(eff, None)
    eff.close()
    return {"dqmc_fp64": {"chains": n, "sweeps": sweeps, "tau_int_sweeps": tau_dq, "ess_per_s": ess_dq,
                          "sweeps_per_s": n * sweeps / t_dq,
                          "local_acceptance": float(acc_dq.sum().item()) / (n * sweeps * N * L)},
            "fit": {"samples": n * sweeps, "terms": len(terms), "r2": float(r2.item())},
            "sldqmc": {"chains": B, "steps": steps, "runs": runs},
            "sldqmc_fp32_chain": run32,
            "sldqmc_learned_action": run_net,
            "burn_in": burn, "ess_ratio": best["ess_per_s"] / ess_dq,
            "ess_ratio_fp32_chain": run32["ess_per_s"] / ess_dq,
            "ess_ratio_learned_action": run_net["ess_per_s"] / ess_dq}


def local_sweep_rate(slq, plan, model, sweeps, seed):
    """Local DQMC sweeps per second on all chains of the plan (one untimed
    sweep first, which also allocates the stabilised partial products)."""
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
    plan = slq.Plan(model, F)
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
    slq.slq_eff_set_net(eff, prm, slq.SLQ_PREC_FP32)
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
    flops = sum(2.0 * m.n_sites ** 3 * (m.n_slices - 1) for m in models)
    info = grp.describe()
    grp.close()
    return {"evals_per_s": 64 / dt, "ms_per_launch": dt * 1e3, "chain_tflops_effective": flops / dt / 1e12,
            "batches": len(info["batches"]), "tuned": info["tuned"]}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--block-width", type=int, default=0,
                    help="vectors per workgroup of the chain-block kernel (0: tuned on the plan)")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-details", action="store_true")
    ap.add_argument("--no-ess", action="store_true",
                    help="skip the effective-samples/s comparison of the two samplers (on by default)")
    ap.add_argument("--ess", action="store_true", help=argparse.SUPPRESS)  # the default; kept for old command lines
    ap.add_argument("--ess-steps", type=int, default=40)
    ap.add_argument("--ess-sweeps", type=int, default=20)
    ap.add_argument("--ess-dqmc-chains", type=int, default=0, help="local-DQMC chains (0: as many as --batch)")
    ap.add_argument("--ess-burn", type=int, default=4)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device to device (a plain copy kernel of known size, against which "
                         "HBM byte counters collected over this run are scaled)")
    ap.add_argument("--sweeps-only", type=int, default=0,
                    help="time this many local DQMC sweeps of --batch chains instead (a profiling aid; "
                         "prints its own JSON line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is a design note.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_1612_03804_amd import slq
    from slq_inputs import DQMC_20x20, iid_fields, default_terms

    if args.copy_calibration:
        src = torch.ones(COPY_CALIBRATION_BYTES // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    model = DQMC_20x20
    B = args.batch
    seed = 0x5D0C + 2
    dev = torch.device("cuda")
    plan = slq.Plan(model, B)
    if args.sweeps_only:
        print(json.dumps(local_sweep_rate(slq, plan, model, args.sweeps_only, seed)), flush=True)
        return
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
    la0, sg0 = logabs.cpu().numpy().copy(), sign.cpu().numpy().copy()

    accepted = torch.zeros((args.warmup + args.steps, B), dtype=torch.int8, device=dev)
    logA = torch.empty(B, dtype=torch.float64, device=dev)
    for w in range(args.warmup):
        slq.slq_cumulative_step(plan, eff, s, logabs, sign, n_moves, seed, w, 0, accepted[w], logA, status)
    torch.cuda.synchronize()

    slq.slq_profile_enable(plan, True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        st = args.warmup + k
        slq.slq_cumulative_step(plan, eff, s, logabs, sign, n_moves, seed, st, 0, accepted[st], logA, status)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gemm_ms, launches, flops = slq.slq_profile_read(plan)
    slq.slq_profile_enable(plan, False)
    elapsed = t1 - t0
    value = B * args.steps / elapsed
    achieved = flops / (gemm_ms * 1e-3) / 1e12 if gemm_ms > 0 else 0.0
    traffic = KRON_TRAFFIC.get(kron_nb) if B == KRON_TRAFFIC_BATCH else None

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
        "data": "synthetic: seeded iid +-1 auxiliary fields, effective model fitted on the GPU",
        "config": {"workload": "dqmc_20x20", "lattice": "20x20", "N": model.n_sites, "L": model.n_slices,
                   "beta": model.beta, "t": model.t, "mu": model.mu, "xi": model.xi, "n_stab": model.n_stab,
                   "chains": B, "effective_moves_per_step": n_moves, "terms": len(terms),
                   "chain_block_vectors_per_workgroup": kron_nb},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": "k_kron: block of 10 slices X <- E diag(d_l) X, E = e^{dtau mu} Cx (x) Cy "
                               "(lattice-line circulant products, FP64 FMA); flops = 2 N^2 (lx+ly) per slice "
                               "and field",
                     "launches": launches, "avg_launch_ms": gemm_ms / max(1, launches),
                     "flops_per_launch": flops / max(1, launches)},
    }

    details = {"fit_r2": float(r2.item()),
               "cumulative_acceptance": float(accepted[args.warmup:].float().mean().item()),
               "chain_kernel_share_of_step": gemm_ms * 1e-3 / elapsed}
    if not args.no_details:
        G = torch.empty((B, model.n_sites, model.n_sites), dtype=torch.float64, device=dev)
        slq.slq_green(plan, s, G, logabs, sign, status)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        slq.slq_green(plan, s, G, logabs, sign, status)
        torch.cuda.synchronize()
        details["green_evals_per_s"] = B / (time.perf_counter() - t0)
        nb = min(B, 64)
        acc = torch.empty(nb, dtype=torch.int64, device=dev)
        drift = torch.empty(nb, dtype=torch.float64, device=dev)
        G2 = G[:nb].clone()
        la2, sg2, st2 = logabs[:nb].clone(), sign[:nb].clone(), status[:nb].clone()
        s2 = s[:nb].clone()
        slq.slq_sweep_local(plan, s2, G2, la2, sg2, 1, seed, 0, 0, acc, drift, st2)  # allocates the stack
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        slq.slq_sweep_local(plan, s[:nb], G[:nb], logabs[:nb], sign[:nb], 1, seed, 0, 0, acc, drift, status[:nb])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        details["dqmc_sweeps_per_s"] = nb / dt
        details["dqmc_chains"] = nb
        details["dqmc_local_acceptance"] = float(acc.sum().item()) / (nb * model.n_sites * model.n_slices)
        details["dqmc_max_drift"] = float(drift.max().item())
        details["group_64_uneven"] = group_rate(slq, dev)
        details["precision_40x40"] = precision_rates(slq)
        details["learned_48x48"] = learned_48x48_rates(slq)
    if not args.no_ess and not args.no_details:
        details["ess"] = ess_rates(slq, plan, model, terms, seed, args.ess_steps, args.ess_dqmc_chains or B,
                                   args.ess_sweeps, args.ess_burn)
    out["details"] = details
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(model, terms, theta_h, fields, la0, sg0, args.cpu_steps, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
