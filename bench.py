"""Benchmark: DIAM chain steps/s and ESS/s on one MI355X, mixed precision vs
plain FP64, Gaussian target d = 4096, P = 256 chains, n_lag = 256.

One benchmark "step" is one window of the sampler: n_lag steps of all P
chains (batched proposal contraction, per-step target contraction and
accept/reject), the moment merge (window scatter) and the refactorisation
(FP64 Cholesky + whitening of the current states).  Inputs are synthetic:
the seeded Gaussian target of the d = 4096 configuration (lambda_i = i^-2,
random orthogonal Q), chains started from exact draws with the global moments
seeded at the target's (warm-start protocol), all random numbers drawn on the
GPU by Philox.  Everything is resident in HBM before timing starts.

Prints ONE JSON line.  ``--gpus N`` with N > 1 is refused: this build runs on
one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ESS/sec and chain steps/sec, d=4096 P=256: mixed-precision vs plain FP64 GPU"
PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15, "fp16": 2.5e15}
HBM_PEAK = 8.0e12
# HBM bytes per launch of the target kernels from rocprofv3 FETCH_SIZE +
# WRITE_SIZE runs scaled by a device copy's counters (see profiles/); a
# kernel missing here has changed since its counters were taken.
# HBM bytes per launch of k_tgt_h2 at d=4096, P=256 (the target's products;
# their K-split reduction runs inside the step kernel k_step_h2), from
# FETCH_SIZE x 2 + WRITE_SIZE (profiles/hbm_traffic_k_tgt_h2_d4096_P256.md);
# taken for the kernel as it stands
TRAFFIC = {"k_tgt_h2": (36902.5 * 2 + 16384.0) * 1024}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def ess_per_chain(traces):
    """Geyer initial-monotone-sequence ESS summed over chains; traces n x P."""
    x = np.asarray(traces, dtype=np.float64)
    n, P = x.shape
    y = x - x.mean(axis=0, keepdims=True)
    m = 1 << int(math.ceil(math.log2(2 * n)))
    f = np.fft.rfft(y, m, axis=0)
    g = np.fft.irfft(f * np.conj(f), m, axis=0)[:n] / n
    tot = 0.0
    for p in range(P):
        gp = g[:, p]
        if gp[0] <= 0:
            continue
        G = gp[0:2 * (n // 2):2] + gp[1:2 * (n // 2):2]
        neg = np.nonzero(G <= 0)[0]
        G = G[:neg[0]] if neg.size else G
        G = np.minimum.accumulate(G)
        tau = max((2.0 * G.sum() - gp[0]) / gp[0], 1.0 / n)
        tot += n / tau
    return tot


def posterior_z_scores(tr, tgt, d, n_lag):
    """z-scores of traced functionals against the target's exact moments:
    log pi = -1/2 chi^2_d (mean -d/2, variance d/2), and v^T x for the
    largest- and smallest-variance eigenvectors (mean v^T mu, variance the
    eigenvalue); tr is steps x 3 x P (log pi, v_max^T x, v_min^T x).  The
    chains share the adapted factor and pivot, so their fluctuations are not
    independent: the standard error comes from batch means, the per-window
    averages over all chains and steps, with the Geyer ESS of that series
    (se).  The figure that treats the chains as independent (the sum of the
    per-chain Geyer ESS) is kept as se_chains / z_chains."""
    out = {}
    truths = (("logpi", -0.5 * d, 0.5 * d), ("v_max", tgt["v_max"] @ tgt["mu"], tgt["lam"][0]),
              ("v_min", tgt["v_min"] @ tgt["mu"], tgt["lam"][-1]))
    worst = worst_chains = 0.0
    nw = tr.shape[0] // n_lag
    for k, (name, mean, var) in enumerate(truths):
        x = tr[:nw * n_lag, k, :]
        for kind, f, truth in (("mean", x, mean), ("variance", (x - mean) ** 2, var)):
            wm = f.reshape(nw, n_lag, -1).mean(axis=(1, 2))
            se = wm.std() / math.sqrt(ess_per_chain(wm[:, None]))
            se_c = f.std() / math.sqrt(ess_per_chain(f))
            z, z_c = (f.mean() - truth) / se, (f.mean() - truth) / se_c
            out[f"{name}_{kind}"] = {"estimate": float(f.mean()), "exact": float(truth), "se": float(se),
                                     "z": float(z), "se_chains": float(se_c), "z_chains": float(z_c)}
            worst = max(worst, abs(z))
            worst_chains = max(worst_chains, abs(z_c))
    out["worst_abs_z"] = worst
    out["worst_abs_z_chains"] = worst_chains
    return out


def run_sampler(prec, tgt, args, torch, diam, profile, stats=False):
    d, P, nl = args.d, args.P, args.n_lag
    dev = torch.device("cuda:0")
    cfg = diam.make_config(d, P, nl, prec, beta=args.beta, seed=args.seed)
    rdt = torch.float64 if prec == "fp64" else torch.float32
    mu = torch.as_tensor(tgt["mu"], device=dev)
    R = torch.as_tensor(tgt["R"], dtype=rdt, device=dev).contiguous()
    x0 = torch.as_tensor(np.ascontiguousarray(tgt["x0"].T), device=dev)
    s = diam.Sampler(cfg, mu, R, x0)
    S0 = torch.as_tensor(tgt["S0"], device=dev)
    m0 = torch.as_tensor(tgt["m0"], device=dev)
    st, _ = s.seed_moments(S0, m0, tgt["N0"])
    assert st == diam.OK
    proj = torch.as_tensor(np.stack([tgt["v_max"], tgt["v_min"]]), device=dev).contiguous()
    n_timed = args.steps * nl
    stat_windows = max(args.steps, getattr(args, "stat_windows", 0) if stats else 0)
    trace = torch.empty((stat_windows * nl, 3, P), dtype=torch.float64, device=dev)

    def window():
        s.step_batch(nl)
        s.merge_moments()
        st, _ = s.update_proposal()
        if st != diam.OK:
            raise RuntimeError(f"update_proposal status {st}")

    for _ in range(args.warmup):
        window()
    torch.cuda.synchronize()
    s.set_trace(proj, trace)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        window()
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    nacc = s.get(diam.F_NACC).view(torch.int32).sum().item()
    # statistics run: the traced windows continue (untimed) to the configured
    # samples per chain, for the posterior-moment z-scores
    t_stat = time.perf_counter()
    for _ in range(stat_windows - args.steps):
        window()
    torch.cuda.synchronize()
    t_stat = time.perf_counter() - t_stat
    s.set_trace(None, None)
    # stopping errors of Section 3.3 (after the timed windows, outside the timing)
    Sig = torch.as_tensor(tgt["S0"] - np.outer(tgt["m0"], tgt["m0"]), device=dev)
    cov_err, mean_err = s.moment_error(Sig, torch.as_tensor(tgt["mu"], device=dev))
    del Sig
    prof = None
    if profile:
        # stage breakdown from HIP events on extra windows (events add small
        # gaps between launches, so they stay out of the timed region)
        s.set_trace(None, None)
        s.profile(True)
        s.profile_read(reset=True)
        s.psrf_enable(True)                      # the PSRF fold is timed in these windows only
        for _ in range(args.profile_windows):
            window()
        prof = s.profile_read(reset=True)
        psrf_worst = s.psrf()[1] if args.profile_windows else None
        s.psrf_enable(False)
        s.profile(False)
    fixed = None
    if stats and getattr(args, "fixed_windows", 0) > 0 and "lam" in tgt:
        # control: the same sampler with the proposal frozen (factor and pivot
        # of the end of the adaptive run; windows are merged but never
        # refactorised), a fixed Metropolis-Hastings kernel whose moments can
        # carry no adaptation bias
        nf = args.fixed_windows
        trf = torch.empty((nf * nl, 3, P), dtype=torch.float64, device=dev)
        s.set_trace(proj, trf)
        nacc_f0 = s.get(diam.F_NACC).view(torch.int32).sum().item()
        for _ in range(nf):
            s.step_batch(nl)
            s.merge_moments()
        torch.cuda.synchronize()
        s.set_trace(None, None)
        acc_f = (s.get(diam.F_NACC).view(torch.int32).sum().item() - nacc_f0) / (P * nl * nf)
        fixed = posterior_z_scores(trf.cpu().numpy(), tgt, d, nl)
        fixed.update(windows=nf, acceptance=acc_f)
        del trf
    tr = trace.cpu().numpy()
    del trace
    half = n_timed // 2
    ess = {name: ess_per_chain(tr[half:n_timed, k, :]) for k, name in enumerate(("logpi", "v_max", "v_min"))}
    moments = None
    if stat_windows > args.steps and "lam" in tgt:
        moments = posterior_z_scores(tr, tgt, d, nl)
        moments.update(windows=stat_windows, samples_per_chain=stat_windows * nl, seconds=T + t_stat)
    del tr
    s.close()
    chain_steps = P * n_timed
    return {
        "seconds": T,
        "chain_steps_per_s": chain_steps / T,
        "steps_per_s": n_timed / T,
        "ms_per_window": 1e3 * T / args.steps,
        # ESS over the second half of the timed run, divided by that half's share of the time
        "ess_per_s": min(ess.values()) / (T * (n_timed - half) / n_timed),
        "ess": ess,
        "acceptance": nacc / (P * (n_timed + args.warmup * nl)),
        "profile": prof,
        "psrf_worst": psrf_worst if profile else None,
        "moments": moments,
        "moments_fixed_proposal": fixed,
        "stopping": {"cov_rel_fro": cov_err, "mean_abs": mean_err, "tol": {"cov_rel_fro": 1e-3, "mean_abs": 1e-2}},
    }


def learned_experiment(args, torch, diam):
    """Learned-part form on the logistic-regression posterior (n = 200000,
    d = 512, P = 128, n_lag = 200): the plain sampler against two-stage
    delayed acceptance with the MLP surrogate trained on the first 5e4 chain
    states.  Both runs start from the same warm start (Laplace mode and
    covariance, host-computed) and run the same collection phase, then the
    same number of timed windows; ESS/s is over the timed windows."""
    from paper_1506_05741_amd import synth
    dev = torch.device("cuda:0")
    d, P, nl = 512, args.learned_P, 200
    t0 = time.perf_counter()
    data = synth.logreg_data()
    mode, C = synth.logreg_laplace(data)
    rng = np.random.default_rng(17)
    Lc = np.linalg.cholesky(C)
    x0 = mode[:, None] + Lc @ rng.standard_normal((d, P))
    ev, V = np.linalg.eigh(C)
    log(f"logistic data + Laplace warm start in {time.perf_counter() - t0:.1f} s")
    A = torch.as_tensor(data.A, device=dev)
    y = torch.as_tensor(data.y, device=dev)
    S0 = torch.as_tensor(C + np.outer(mode, mode), device=dev)
    m0 = torch.as_tensor(mode, device=dev)
    proj = torch.as_tensor(np.stack([V[:, -1], V[:, 0]]), device=dev).contiguous()
    n_pairs = 50000
    collect = -(-n_pairs // P)                            # steps whose states train the surrogate
    # (beta, alpha) settings: the step size and the inflation of eq. diamnl
    settings = [tuple(float(v) for v in pair.split(":")) if ":" in pair else (float(pair), 1.0)
                for pair in args.learned_settings.split(",")]
    out = {"workload": f"Bayesian logistic regression n=200000 d={d} (A ~ N(0, 1/d), prior N(0, 10 I)), "
                       f"P={P}, n_lag={nl}, Laplace warm start; surrogate form {args.surrogate_form}",
           "precision": args.learned_precision, "runs": []}
    for (beta, alpha), use_da in [(st, u) for st in settings for u in (False, True)]:
        cfg = diam.make_config(d, P, nl, args.learned_precision, beta=beta, alpha=alpha, seed=91,
                               surrogate=args.surrogate_form if use_da else 0, train_max=n_pairs)
        s = diam.Sampler(cfg, None, None, torch.as_tensor(np.ascontiguousarray(x0.T), device=dev), A=A, y=y,
                         prior_var=data.prior_var)
        assert s.seed_moments(S0, m0, 10 * P * nl)[0] == diam.OK
        Xtr = torch.empty((collect * P, d), dtype=torch.float64, device=dev)
        ltr = torch.empty(collect * P, dtype=torch.float64, device=dev)
        done = 0
        while done < collect:                             # collection phase, identical in both runs
            k = min(collect - done, nl - s.stats()["steps_in_window"])
            for _ in range(k):
                s.step_batch(1)
                Xtr[done * P:(done + 1) * P] = s.get_f64(diam.F_X, (P, d))
                ltr[done * P:(done + 1) * P] = s.get_f64(diam.F_LOGP, (P,))
                done += 1
            if s.stats()["steps_in_window"] == nl:
                s.merge_moments()
                assert s.update_proposal()[0] == diam.OK
        rest = nl - s.stats()["steps_in_window"]          # finish the window
        if rest:
            s.step_batch(rest)
            s.merge_moments()
            assert s.update_proposal()[0] == diam.OK
        train_s = None
        if use_da:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            loss = s.surrogate_train(Xtr[:n_pairs], ltr[:n_pairs], steps=args.train_steps, batch=256, lr=1e-3,
                                     seed=5)
            s.set_delayed_acceptance(True)
            torch.cuda.synchronize()
            train_s = time.perf_counter() - t1
            surr = {"pairs": n_pairs, "adam_steps": args.train_steps, "batch": 256, "final_loss": loss,
                    "train_seconds": train_s}
        n_timed = args.learned_windows * nl
        trace = torch.empty((n_timed, 3, P), dtype=torch.float64, device=dev)
        s.set_trace(proj, trace)
        nacc0 = s.get(diam.F_NACC).view(torch.int32).sum().item()
        npass0 = s.get(diam.F_NPASS).view(torch.int32).sum().item() if use_da else 0
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.learned_windows):
            s.step_batch(nl)
            s.merge_moments()
            assert s.update_proposal()[0] == diam.OK
        torch.cuda.synchronize()
        T = time.perf_counter() - t1
        tr = trace.cpu().numpy()
        nacc = s.get(diam.F_NACC).view(torch.int32).sum().item() - nacc0
        npass = (s.get(diam.F_NPASS).view(torch.int32).sum().item() - npass0) if use_da else 0
        s.set_trace(None, None)
        s.profile(True)
        s.profile_read(reset=True)
        s.step_batch(nl)
        s.merge_moments()
        assert s.update_proposal()[0] == diam.OK
        prof = s.profile_read(reset=True)
        s.profile(False)
        ess = {name: ess_per_chain(tr[:, k, :]) for k, name in enumerate(("logpi", "v_max", "v_min"))}
        r = {"beta": beta, "alpha": alpha, "delayed_acceptance": use_da,
             "seconds": T, "chain_steps_per_s": P * n_timed / T, "ess": ess, "ess_per_s": min(ess.values()) / T,
             "acceptance": nacc / (P * n_timed),
             "stage_ms_per_window": {k: v[0] for k, v in prof.items() if v[1]}}
        if use_da:
            r["stage1_pass_rate"] = npass / (P * n_timed)
            r["stage2_accept_rate"] = nacc / max(npass, 1)
            r["ess_per_s_incl_training"] = min(ess.values()) / (T + train_s)
            r["surrogate"] = surr
        out["runs"].append(r)
        log(f"logistic beta={beta} alpha={alpha} {'DA' if use_da else 'plain'}: "
            f"{r['chain_steps_per_s']:.4g} chain-steps/s, "
            f"ESS/s {r['ess_per_s']:.4g}, acceptance {r['acceptance']:.3f}"
            + (f", stage-1 pass {r['stage1_pass_rate']:.3f}" if use_da else ""))
        s.close()
        del Xtr, ltr, trace
    plain = {(r["beta"], r["alpha"]): r for r in out["runs"] if not r["delayed_acceptance"]}
    da = {(r["beta"], r["alpha"]): r for r in out["runs"] if r["delayed_acceptance"]}
    out["ess_per_s_gain_at_setting"] = {f"beta={b},alpha={a}": da[(b, a)]["ess_per_s"] / plain[(b, a)]["ess_per_s"]
                                        for b, a in settings}
    # what the network does per exact evaluation: ESS per exact target evaluation, DA / plain
    out["ess_per_exact_eval_gain_at_setting"] = {
        f"beta={b},alpha={a}": (min(da[(b, a)]["ess"].values()) / (da[(b, a)]["stage1_pass_rate"]))
        / min(plain[(b, a)]["ess"].values()) for b, a in settings}
    best_plain = max(r["ess_per_s"] for r in plain.values())
    best_da = max(r["ess_per_s"] for r in da.values())
    out["best_plain_ess_per_s"] = best_plain
    out["best_da_ess_per_s"] = best_da
    out["ess_per_s_gain"] = best_da / best_plain
    return out


def batch_experiment(args, torch, diam):
    """Batched form: 48 independent Gaussian targets, d log-uniform in
    [128, 3072] (lambda_i = i^-2, seed 1000 + g), 32 chains each, n_lag = 128,
    FP32 with FP64 Cholesky, warm start.  One benchmark window = n_lag steps
    of all 1536 chains + merge + refactorisation of all 48 problems (grouped
    launches, graph-captured window), against the same windows run problem by
    problem through the single-problem API."""
    from paper_1506_05741_amd import synth
    dev = torch.device("cuda:0")
    P, nl = 32, 128
    dims = [int(x) for x in synth.batch_dims(48)]
    t0 = time.perf_counter()
    ts = [synth.gaussian_target(d, 1000 + g) for g, d in enumerate(dims)]
    x0 = [synth.gaussian_exact_draws(t, P, 2000 + g) for g, t in enumerate(ts)]
    log(f"48 batch targets built in {time.perf_counter() - t0:.1f} s")
    mus = [torch.as_tensor(t.mu, device=dev) for t in ts]
    Rs = [torch.as_tensor(t.R, dtype=torch.float32, device=dev).contiguous() for t in ts]
    xs = [torch.as_tensor(np.ascontiguousarray(x.T), device=dev) for x in x0]
    S0 = [torch.as_tensor(t.Sigma + np.outer(t.mu, t.mu), device=dev) for t in ts]
    m0 = [torch.as_tensor(t.mu, device=dev) for t in ts]
    # warm start with N0 = P x the run's samples per chain (100 windows of 128
    # steps): with only 10 windows the adaptation at d ~ 3000 degrades the
    # acceptance and the window-end variances within tens of windows
    N0 = float(P) * 12800
    cfg = diam.make_batch_config(48, P, nl, beta=0.3, seed=77)
    b = diam.Batch(cfg, mus, Rs, xs)
    assert b.seed_moments(S0, m0, N0)[0] == diam.OK
    choice, us = b.autotune(reps=20)
    for _ in range(1):
        assert b.window()[0] == diam.OK
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.batch_windows):
        st, _ = b.window()
        assert st == diam.OK
    torch.cuda.synchronize()
    T = time.perf_counter() - t1
    nacc = sum(int(b.get(g, diam.F_NACC).view(torch.int32).sum()) for g in range(48))
    acc = nacc / (48 * P * nl * (args.batch_windows + 1))
    # ESS and per-target moments from window-end states of further, untimed
    # windows: projections on each target's largest- and smallest-variance
    # eigenvectors; ESS per window (minimum of the two) summed over the 48
    # targets, times the timed windows per second
    proj = [np.stack([t.Q[:, 0], t.Q[:, -1]]) for t in ts]
    series = [[] for _ in ts]
    for _ in range(args.batch_ess_windows):
        assert b.window()[0] == diam.OK
        for g, t in enumerate(ts):
            series[g].append(b.get_f64(g, diam.F_X, (P, t.d)).cpu().numpy() @ proj[g].T)
    ess_win, worst, worst_at = 0.0, 0.0, None
    for g, t in enumerate(ts):
        Y = np.stack(series[g])                               # windows x P x 2
        es = []
        for f, lam in ((0, t.lam[0]), (1, t.lam[-1])):
            y, m = Y[:, :, f], proj[g][f] @ t.mu
            es.append(ess_per_chain(y))
            for kind, h, truth in (("mean", y, m), ("variance", (y - m) ** 2, lam)):
                z = (h.mean() - truth) / (h.std() / math.sqrt(ess_per_chain(h)))
                if abs(z) > worst:
                    worst = abs(z)
                    worst_at = {"target": g, "d": t.d, "functional": ("v_max" if f == 0 else "v_min") + "^T x",
                                "moment": kind, "z": float(z)}
        ess_win += min(es) / Y.shape[0]
    b.close()
    chain_steps = 48 * P * nl * args.batch_windows
    flops = 2.0 * sum(d * d for d in dims) * P
    out = {"workload": "48 Gaussian targets, d log-uniform in [128, 3072] (sum d = %d), 32 chains each, "
                       "n_lag=128, beta=0.3, fp32 with fp64 Cholesky, warm start N0=32*12800" % sum(dims),
           "windows": args.batch_windows, "ms_per_window": 1e3 * T / args.batch_windows,
           "chain_steps_per_s": chain_steps / T, "acceptance": acc,
           "ess_per_s_summed": ess_win * args.batch_windows / T,
           "ess": {"windows": args.batch_ess_windows, "per_window_summed": ess_win,
                   "worst_z_moments": worst, "worst": worst_at,
                   "note": "window-end states of the 48 targets, v_max^T x and v_min^T x; worst |z| of their "
                           "means and variances against the exact values over all targets"},
           "autotune_us_per_target_launch": us, "tile_choice": diam.BATCH_TILES[choice],
           "target_roofline": {"kernel": "gk_tgt (grouped fp32 MFMA target contraction)", "bound": "mfma",
                               "achieved": flops / (us[diam.BATCH_TILES[choice]] * 1e-6) / 1e12,
                               "peak": PEAK["fp32"] / 1e12, "unit": "TFLOP/s",
                               "frac": flops / (us[diam.BATCH_TILES[choice]] * 1e-6) / PEAK["fp32"]}}
    # the same windows with the n_lag loop as one persistent launch (a device
    # queue of (problem, phase, tile) items; default 64 x 2 target tiles)
    bp = diam.Batch(cfg, mus, Rs, xs)
    assert bp.seed_moments(S0, m0, N0)[0] == diam.OK
    bp.set_persistent(True)
    assert bp.window()[0] == diam.OK
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.batch_windows):
        st, _ = bp.window()
        assert st == diam.OK
    torch.cuda.synchronize()
    Tp = time.perf_counter() - t1
    bp.close()
    out["persistent"] = {"windows": args.batch_windows, "ms_per_window": 1e3 * Tp / args.batch_windows,
                         "chain_steps_per_s": chain_steps / Tp, "vs_graph": T / Tp,
                         "note": "the n_lag loop of every window as one persistent launch over a device work "
                                 "queue, graph-captured window, default 64x2 target tiles"}
    # the same windows problem by problem through the single-problem API
    singles = []
    for g, t in enumerate(ts):
        c = diam.make_config(t.d, P, nl, "fp32", beta=0.3, seed=77 + g)
        s = diam.Sampler(c, mus[g], Rs[g], xs[g])
        assert s.seed_moments(S0[g], m0[g], N0)[0] == diam.OK
        singles.append(s)

    def seq_window():
        for s in singles:
            s.step_batch(nl)
            s.merge_moments()
            assert s.update_proposal()[0] == diam.OK

    seq_window()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nseq = max(1, args.batch_windows // 2)
    for _ in range(nseq):
        seq_window()
    torch.cuda.synchronize()
    Ts = time.perf_counter() - t1
    for s in singles:
        s.close()
    out["sequential"] = {"windows": nseq, "ms_per_window": 1e3 * Ts / nseq,
                         "chain_steps_per_s": 48 * P * nl * nseq / Ts}
    out["speedup_vs_sequential"] = out["chain_steps_per_s"] / out["sequential"]["chain_steps_per_s"]
    log(f"batch: {out['chain_steps_per_s']:.4g} chain-steps/s ({out['ms_per_window']:.2f} ms/window, tiles "
        f"{out['tile_choice']}), persistent loop {out['persistent']['ms_per_window']:.2f} ms/window, sequential "
        f"{out['sequential']['chain_steps_per_s']:.4g}, ESS/s summed {out['ess_per_s_summed']:.4g}, "
        f"worst |z| {worst:.2f} ({out['ess']['worst']})")
    return out


FAMILY_BANDS = {"diam": (0.3, 0.5), "am": (0.1, 0.3), "pcn": (0.3, 0.5), "rw": (0.1, 0.3)}


def families_experiment(args, torch, diam):
    """Section 3.2's comparison (its Fig. 1) through the same kernels: DIAM,
    AM, pCN and RW on pi_1, pi_2, pi_4 (data variance 1/d and 1/d^2) and pi_5
    (alpha = 1.2) at d = 100, 32 chains, n_lag = 100, FP64, beta adapted from
    2.4/sqrt(d) inside each family's acceptance band.  DIAM and AM start from
    the exact moments (warm start); pCN and RW keep A = I, x_ref = 0.  The
    second half of the run is traced and timed: ESS of log pi, v_d^T x and
    v_1^T x, ESS/s = the minimum over the three / time of the traced windows."""
    from paper_1506_05741_amd import synth
    d, P, nl, W = 100, 32, 100, args.family_windows
    half = W // 2
    dev = torch.device("cuda:0")
    out = {"workload": f"Section 3.2 comparison: d={d}, P={P}, n_lag={nl}, {W} windows (last {W - half} traced), "
                       "fp64, beta adapted from 2.4/sqrt(d)", "targets": {}}
    for tgt in ("pi1", "pi2", "pi4", "pi4s", "pi5"):
        twist, alpha = None, 1.0
        if tgt == "pi5":
            tw = synth.twisted_target(d, 1, 0.3)
            R, mu, twist, V = tw.R, tw.mu, tw.c, tw.V
            x0 = synth.twisted_exact_draws(tw, P, 2)
            S0, m0 = synth.twisted_warm_moments(tw)
            v_d, v_1, alpha = V[:, -1], V[:, 0], 1.2
        else:
            name, s2 = ("pi4", 1.0 / d ** 2) if tgt == "pi4s" else (tgt, None)
            t = synth.paper_gaussian(name, d, 1, s2)
            R, mu = t.R, t.mu
            x0 = synth.gaussian_exact_draws(t, P, 2)
            S0, m0 = synth.gaussian_warm_moments(t)
            v_d, v_1 = t.v_max, t.v_min
        rows = {}
        for prop in ("diam", "am", "pcn", "rw"):
            band = FAMILY_BANDS[prop]
            cfg = diam.make_config(d, P, nl, "fp64", beta=2.4 / math.sqrt(d), alpha=alpha, seed=31, proposal=prop)
            smp = diam.Sampler(cfg, torch.as_tensor(mu, device=dev), torch.as_tensor(R, device=dev),
                               torch.as_tensor(np.ascontiguousarray(x0.T), device=dev),
                               twist=None if twist is None else torch.as_tensor(twist, device=dev))
            smp.set_beta_adaptation(True, band[0], band[1], 1.2, 1.0)
            if prop in ("diam", "am"):
                assert smp.seed_moments(torch.as_tensor(S0, device=dev), torch.as_tensor(m0, device=dev),
                                        10.0 * P * nl)[0] == diam.OK
            for _ in range(half):
                smp.step_batch(nl)
                smp.merge_moments()
                assert smp.update_proposal()[0] == diam.OK
            trace = torch.zeros(((W - half) * nl, 3, P), dtype=torch.float64, device=dev)
            smp.set_trace(torch.as_tensor(np.stack([v_d, v_1]), device=dev), trace)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(W - half):
                smp.step_batch(nl)
                smp.merge_moments()
                assert smp.update_proposal()[0] == diam.OK
            torch.cuda.synchronize()
            T = time.perf_counter() - t1
            tr = trace.cpu().numpy()
            ess = [ess_per_chain(tr[:, f, :]) for f in range(3)]
            rows[prop] = {"ess_per_s": min(ess) / T, "ess_per_step": [e / tr.shape[0] for e in ess],
                          "chain_steps_per_s": P * nl * (W - half) / T, "beta": smp.stats()["beta"]}
            smp.close()
        out["targets"][tgt] = rows
        log(f"families {tgt}: " + ", ".join(f"{k} {v['ess_per_s']:.4g} ESS/s" for k, v in rows.items()))
    return out


def precision_experiment(args, torch, diam):
    """The d = 1024 configuration: Gaussian target seed 1 (lambda_i = i^-2,
    cond 1.05e6), P = 64, n_lag = 200, beta = 0.3, warm start with N0 = P 1e5;
    FP64 against FP32 (and the mixed form), each timed over whole windows with
    ESS over the second half."""
    import argparse as _ap
    from paper_1506_05741_amd import synth
    d, P, nl = 1024, 64, 200
    t = synth.gaussian_target(d, 1)
    x0 = synth.gaussian_exact_draws(t, P, 2)
    S0, m0 = synth.gaussian_warm_moments(t)
    tgt = dict(mu=t.mu, R=t.R, x0=x0, S0=S0, m0=m0, N0=float(P) * 1e5, v_max=t.v_max, v_min=t.v_min)
    sub = _ap.Namespace(**vars(args))
    sub.d, sub.P, sub.n_lag, sub.beta, sub.steps, sub.warmup = d, P, nl, 0.3, args.c2_windows, 2
    out = {"workload": f"Gaussian d={d} (seed 1), P={P}, n_lag={nl}, beta=0.3, warm start N0=P*1e5; "
                       f"{args.c2_windows} timed windows", "precisions": {}}
    for prec in ("fp64", "fp32", "mixed"):
        r = run_sampler(prec, tgt, sub, torch, diam, profile=False)
        out["precisions"][prec] = {k: r[k] for k in ("chain_steps_per_s", "ess_per_s", "ms_per_window", "acceptance")}
        log(f"d=1024 {prec}: {r['chain_steps_per_s']:.4g} chain-steps/s, ESS/s {r['ess_per_s']:.4g}, "
            f"{r['ms_per_window']:.2f} ms/window")
    f64 = out["precisions"]["fp64"]
    out["speedup_vs_fp64"] = {p: {"chain_steps": v["chain_steps_per_s"] / f64["chain_steps_per_s"],
                                  "ess": v["ess_per_s"] / f64["ess_per_s"]}
                              for p, v in out["precisions"].items() if p != "fp64"}
    return out


def local_global_experiment(args, torch, diam):
    """Section 2.4.1's logistics with M intervals per batch: M = 1 (every
    merge global, one shared factor) against M = 4 (each chain refactorised
    from its local update of the global moments between global merges), FP64,
    Gaussian target d = 1024 (seed 1, lambda_i = i^-2), P = 64, n_lag = 200,
    warm start with N0 = P 1e5 as the d = 1024 configuration.  Timed: whole batches (one window = one
    interval); the stage split comes from HIP events on one further batch."""
    from paper_1506_05741_amd import synth
    d, P, nl = 1024, 64, 200
    dev = torch.device("cuda:0")
    t = synth.gaussian_target(d, 1)
    x0 = torch.as_tensor(np.ascontiguousarray(synth.gaussian_exact_draws(t, P, 2).T), device=dev)
    S0, m0 = synth.gaussian_warm_moments(t)
    mu, R = torch.as_tensor(t.mu, device=dev), torch.as_tensor(t.R, device=dev)
    proj = torch.as_tensor(np.stack([t.v_max, t.v_min]), device=dev).contiguous()
    out = {"workload": f"Gaussian d={d} (seed 1), P={P}, n_lag={nl}, fp64, beta=0.3, warm start N0=P*1e5; "
                       "window = one interval of n_lag steps", "M": {}}
    for M in (1, 4):
        smp = diam.Sampler(diam.make_config(d, P, nl, "fp64", beta=0.3, seed=41, M=M), mu, R, x0)
        assert smp.seed_moments(torch.as_tensor(S0, device=dev), torch.as_tensor(m0, device=dev),
                                float(P) * 1e5)[0] == diam.OK

        def window():
            smp.step_batch(nl)
            smp.merge_moments()
            assert smp.update_proposal()[0] == diam.OK

        for _ in range(4):
            window()
        nwin = args.lg_windows
        trace = torch.empty((nwin * nl, 3, P), dtype=torch.float64, device=dev)
        smp.set_trace(proj, trace)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(nwin):
            window()
        torch.cuda.synchronize()
        T = time.perf_counter() - t1
        smp.set_trace(None, None)
        smp.profile(True)
        smp.profile_read(reset=True)
        for _ in range(4):
            window()
        prof = smp.profile_read(reset=True)
        smp.profile(False)
        tr = trace.cpu().numpy()
        ess = [ess_per_chain(tr[:, f, :]) for f in range(3)]
        out["M"][str(M)] = {"windows": nwin, "ms_per_window": 1e3 * T / nwin,
                            "chain_steps_per_s": P * nl * nwin / T, "ess_per_s": min(ess) / T,
                            "stage_ms_per_window": {k: v[0] / 4 for k, v in prof.items() if v[1]}}
        smp.close()
        log(f"local-global M={M}: {out['M'][str(M)]['ms_per_window']:.2f} ms/window, "
            f"{out['M'][str(M)]['ess_per_s']:.4g} ESS/s")
    return out


def host_info():
    """The host the oracle runs on: core count, CPU model, NumPy's BLAS
    backend and the threads its pool uses."""
    info = {"cpu_count": os.cpu_count(), "cpu_model": None, "blas": None, "blas_threads": None}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        blas = np.show_config(mode="dicts")["Build Dependencies"]["blas"]
        info["blas"] = f"{blas.get('name')} {blas.get('version', '')}".strip()
    except Exception:
        pass
    try:
        from threadpoolctl import threadpool_info
        pools = [p for p in threadpool_info() if p.get("user_api") == "blas"]
        if pools:
            info["blas_threads"] = max(int(p.get("num_threads", 1)) for p in pools)
            info["blas"] = info["blas"] or pools[0].get("internal_api")
    except Exception:
        pass
    return info


def _oracle_windows(o, d, P, nl, windows, seed):
    """Time `windows` whole windows of the oracle (steps, merge, update) on
    seeded normals and uniforms drawn outside the timing."""
    from paper_1506_05741_amd import synth
    T = 0.0
    for w in range(windows):
        W = synth.draw_normals(d, P, nl, seed + 2 * w)
        U = synth.draw_uniforms(P, nl, seed + 2 * w + 1)
        t0 = time.perf_counter()
        for t in range(nl):
            o.step(W[t].T, U[t])
        o.merge_moments()
        o.update_proposal()
        T += time.perf_counter() - t0
    return T


def cpu_baseline(tgt, args):
    """The FP64 oracle on the host cores.  The d = 4096 workload (the line's
    unit): a bounded sample of a few steps of all P chains, one merge of those
    steps (scaled to a window's length) and one refactorisation, extrapolated
    to whole windows; two full windows would take about half an hour.  The
    d = 32 configuration as a full run (400 windows, literal cold start) and
    the d = 1024 configuration over two whole windows (warm start), both
    timed directly."""
    from oracle import diam as od
    from oracle import targets as ot
    from paper_1506_05741_amd import synth
    info = host_info()
    cores = info["blas_threads"] or info["cpu_count"]
    d, P, nl = args.d, args.P, args.n_lag
    R, mu = tgt["R"], tgt["mu"]
    o = od.DiamOracle(lambda X: ot.gaussian_logpdf(R, mu, X), d, P, nl, args.beta, X=tgt["x0"])
    o.seed_moments(tgt["S0"], tgt["m0"], tgt["N0"])
    ns = args.cpu_steps
    W = synth.draw_normals(d, P, ns, 11)
    U = synth.draw_uniforms(P, ns, 12)
    t0 = time.perf_counter()
    for t in range(ns):
        o.step(W[t].T, U[t])
    t_step = (time.perf_counter() - t0) / ns
    t0 = time.perf_counter()
    o.merge_moments()
    t_merge = (time.perf_counter() - t0) * nl / ns       # the scatter scales with the window length
    t0 = time.perf_counter()
    o.update_proposal()
    t_update = time.perf_counter() - t0
    t_window = nl * t_step + t_merge + t_update
    del o
    configs = {}
    # d = 32, P = 4, n_lag = 50, 2e4 samples per chain: the whole run
    t32 = synth.gaussian_target(32, 0)
    o32 = od.DiamOracle(lambda X: ot.gaussian_logpdf(t32.R, t32.mu, X), 32, 4, 50, 0.3, X=np.zeros((32, 4)))
    T32 = _oracle_windows(o32, 32, 4, 50, 400, 1000)
    configs["d32"] = {"chain_steps_per_s": 4 * 50 * 400 / T32, "seconds": T32,
                      "run": "full: 400 windows of 50 steps, P = 4, literal cold start"}
    # d = 1024, P = 64, n_lag = 200: two whole windows from the warm start
    t1k = synth.gaussian_target(1024, 1)
    S1, m1 = synth.gaussian_warm_moments(t1k)
    o1k = od.DiamOracle(lambda X: ot.gaussian_logpdf(t1k.R, t1k.mu, X), 1024, 64, 200, 0.3,
                        X=synth.gaussian_exact_draws(t1k, 64, 2))
    o1k.seed_moments(S1, m1, 64 * 1e5)
    T1k = _oracle_windows(o1k, 1024, 64, 200, 2, 2000)
    configs["d1024"] = {"chain_steps_per_s": 64 * 200 * 2 / T1k, "seconds": T1k,
                        "run": "2 whole windows of 200 steps, P = 64, warm start"}
    return {
        "value": P * nl / t_window, "unit": "chain-steps/s", "cores": cores, "kind": "oracle",
        "sample": f"{ns} steps of all {P} chains at d={d}, one merge of those steps scaled to n_lag={nl}, "
                  f"one FP64 refactorisation; per window {t_window:.1f} s (extrapolated)",
        "host": info, "configs": configs,
        "note": "NumPy FP64 oracle with the plain triangular solve for z (d^2 P more flops per step than "
                "the GPU's recurrence); ESS/s(oracle) = its steps/s x the GPU run's ESS per step",
    }


def library_gemm_reference(d, P, torch):
    """The vendor GEMM (torch.matmul on hipBLASLt) at the target's shape, for
    context beside the roofline: one f16 product R V (d x d by d x P, FP32
    accumulation inside) and the three-product form as one product of K = 3 d
    ([R1 R0 R0] by [V0; V1; V0])."""
    out = {}
    for name, k in (("one_f16_product", d), ("three_products_as_K_3d", 3 * d)):
        a = torch.randn(d, k, device="cuda").to(torch.float16)
        b = torch.randn(k, P, device="cuda").to(torch.float16)
        for _ in range(5):
            c = a @ b
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(50):
            c = a @ b
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / 50 * 1e3
        out[name] = {"us": us, "tflops": 2.0 * d * k * P / (us * 1e-6) / 1e12}
        del a, b, c
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=12, help="timed windows")
    ap.add_argument("--warmup", type=int, default=2, help="untimed windows")
    ap.add_argument("--fixed-windows", dest="fixed_windows", type=int, default=196,
                    help="traced windows with the proposal frozen after the statistics run (0: none)")
    ap.add_argument("--stat-windows", dest="stat_windows", type=int, default=196,
                    help="traced windows (timed ones included) for the posterior-moment z-scores: 196 windows = "
                         "5e4 samples per chain at n_lag = 256")
    ap.add_argument("--d", type=int, default=4096)
    ap.add_argument("--P", type=int, default=256)
    ap.add_argument("--n-lag", dest="n_lag", type=int, default=256)
    ap.add_argument("--beta", type=float, default=0.3)
    ap.add_argument("--seed", type=int, default=2026)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp32", "fp64"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=16)
    ap.add_argument("--profile-windows", dest="profile_windows", type=int, default=2,
                    help="extra windows timed per stage with HIP events (after the timed region)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-part (logistic) experiment")
    ap.add_argument("--copy-calibration", dest="copy_calibration", type=int, default=0,
                    help="first run 3 device copies of this many bytes (counter calibration)")
    ap.add_argument("--learned-only", action="store_true", help="run only the learned-part experiment")
    ap.add_argument("--learned-P", dest="learned_P", type=int, default=128)
    ap.add_argument("--learned-settings", dest="learned_settings", default="0.5,1.0,1.0:1.2,1.0:1.5",
                    help="comma-separated beta or beta:alpha settings of the learned-form comparison")
    ap.add_argument("--surrogate-form", dest="surrogate_form", type=int, default=2, choices=[1, 2])
    ap.add_argument("--learned-windows", dest="learned_windows", type=int, default=4)
    ap.add_argument("--learned-precision", dest="learned_precision", default="fp32", choices=["mixed", "fp32", "fp64"])
    ap.add_argument("--train-steps", dest="train_steps", type=int, default=3000)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-form experiment")
    ap.add_argument("--batch-only", action="store_true", help="run only the batched-form experiment")
    ap.add_argument("--batch-windows", dest="batch_windows", type=int, default=6)
    ap.add_argument("--batch-ess-windows", dest="batch_ess_windows", type=int, default=40)
    ap.add_argument("--no-families", action="store_true", help="skip the proposal-family comparison")
    ap.add_argument("--families-only", action="store_true", help="run only the proposal-family comparison")
    ap.add_argument("--family-windows", dest="family_windows", type=int, default=120)
    ap.add_argument("--no-local-global", action="store_true", help="skip the M > 1 logistics experiment")
    ap.add_argument("--local-global-only", action="store_true", help="run only the M > 1 logistics experiment")
    ap.add_argument("--lg-windows", dest="lg_windows", type=int, default=8)
    ap.add_argument("--no-d1024", action="store_true", help="skip the d = 1024 precision comparison")
    ap.add_argument("--d1024-only", action="store_true", help="run only the d = 1024 precision comparison")
    ap.add_argument("--c2-windows", dest="c2_windows", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported by this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1506_05741_amd import diam, synth
    diam.load()
    if args.copy_calibration:
        # a plain device copy of known size: its FETCH_SIZE / WRITE_SIZE
        # counters calibrate the kernel's HBM traffic figures
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {n * 4} bytes")
        del src, dst

    if args.batch_only:
        print(json.dumps({"batch": batch_experiment(args, torch, diam)}), flush=True)
        return
    if args.learned_only:
        print(json.dumps({"learned": learned_experiment(args, torch, diam)}), flush=True)
        return
    if args.families_only:
        print(json.dumps({"families": families_experiment(args, torch, diam)}), flush=True)
        return
    if args.d1024_only:
        print(json.dumps({"d1024": precision_experiment(args, torch, diam)}), flush=True)
        return
    if args.local_global_only:
        print(json.dumps({"local_global": local_global_experiment(args, torch, diam)}), flush=True)
        return

    # -- synthetic workload (host), seeded as the d = 4096 configuration ------
    t0 = time.perf_counter()
    t = synth.gaussian_target(args.d, 2)
    x0 = synth.gaussian_exact_draws(t, args.P, 3)
    S0, m0 = synth.gaussian_warm_moments(t)
    tgt = dict(mu=t.mu, R=t.R, x0=x0, S0=S0, m0=m0, N0=float(args.P) * 50176,
               v_max=t.v_max, v_min=t.v_min, lam=t.lam)
    log(f"target built in {time.perf_counter() - t0:.1f} s")

    res = run_sampler(args.precision, tgt, args, torch, diam, profile=True, stats=True)
    log(f"{args.precision}: {res['chain_steps_per_s']:.4g} chain-steps/s, ESS/s {res['ess_per_s']:.4g}, "
        f"{res['ms_per_window']:.2f} ms/window, acceptance {res['acceptance']:.3f}")
    ref = None
    if not args.no_fp64 and args.precision != "fp64":
        ref = run_sampler("fp64", tgt, args, torch, diam, profile=True, stats=True)
        log(f"fp64: {ref['chain_steps_per_s']:.4g} chain-steps/s, ESS/s {ref['ess_per_s']:.4g}, "
            f"{ref['ms_per_window']:.2f} ms/window")

    # -- roofline of the dominant kernel: the per-step target contraction -----
    prof = res["profile"]
    ms_t, n_t = prof["target"]
    useful = 2.0 * args.d * args.d * args.P          # algorithmic flops of Y = R (x - mu) per step
    dt = (ms_t / n_t) * 1e-3
    split = args.precision == "mixed" and args.d % 128 == 0 and args.P % 64 == 0
    method_bytes = 4.0 * args.d * args.d + 4.0 * args.d * args.P    # R (FP32) and x - mu read once
    if split:
        # two half parts per operand, three half products per FP32-equivalent
        # product: frac counts the method's 2 d^2 P flops, executed_frac the
        # three products the matrix cores run
        traffic = TRAFFIC.get("k_tgt_h2") if (args.d, args.P) == (4096, 256) else None
        roofline = {"kernel": "k_tgt_h2 (two-part half MFMA, FP32-equivalent; Y = R (x - mu) as four K-split "
                              "partials, reduced and squared inside the step kernel k_step_h2)",
                    "bound": "mfma", "achieved": useful / dt / 1e12, "peak": PEAK["fp16"] / 1e12,
                    "unit": "TFLOP/s", "frac": useful / dt / PEAK["fp16"],
                    "traffic": traffic,
                    "traffic_ratio": (traffic / method_bytes) if traffic else None,
                    "method_bytes": method_bytes,
                    "executed_tflops": 3 * useful / dt / 1e12, "executed_frac": 3 * useful / dt / PEAK["fp16"],
                    "fp32_equivalent_frac": useful / dt / PEAK["fp32"],
                    "avg_us": dt * 1e6, "launches": n_t,
                    "work": "2 d^2 P flops per step (useful); 3 x that in half products executed"}
    else:
        tdt = "fp64" if args.precision == "fp64" else "fp32"
        roofline = {"kernel": f"k_tgt_gauss ({tdt} MFMA, Y = R (x - mu), column sums of Y^2)",
                    "bound": "mfma", "achieved": useful / dt / 1e12, "peak": PEAK[tdt] / 1e12, "unit": "TFLOP/s",
                    "frac": useful / dt / PEAK[tdt], "traffic": TRAFFIC.get(f"k_tgt_gauss_{tdt}"),
                    "avg_us": dt * 1e6, "launches": n_t}
    # the proposal contraction of the window (aimed at 60 % or more of the
    # bf16 peak): frac on the triangular d (d + 1) P n_lag flops of the method,
    # executed_frac on the four bf16 hi/lo products the matrix cores run
    ms_p, n_p = prof["proposal"]
    if args.precision == "mixed" and n_p:
        pf = float(args.d) * (args.d + 1) * args.P * args.n_lag
        dtp = ms_p / n_p * 1e-3
        roofline["proposal"] = {"kernel": "k_trigemm_hl (bf16 hi/lo, direct-to-LDS)", "achieved": pf / dtp / 1e12,
                                "peak": PEAK["bf16"] / 1e12, "unit": "TFLOP/s", "frac": pf / dtp / PEAK["bf16"],
                                "executed_tflops": 4 * pf / dtp / 1e12, "executed_frac": 4 * pf / dtp / PEAK["bf16"],
                                "avg_us": dtp * 1e6,
                                "work": "d (d + 1) P n_lag flops per window (useful, triangular); 4 x that executed"}
    if args.precision == "mixed" and split:
        roofline["library_reference"] = library_gemm_reference(args.d, args.P, torch)
    stages = {k: {"ms_per_window": v[0] / args.profile_windows, "regions": v[1]} for k, v in prof.items() if v[1]}
    # the PSRF fold of a merged window (profiled windows only): store read + accumulators read and written
    psrf = None
    ms_ps, n_ps = prof.get("psrf", (0.0, 0))
    if n_ps:
        eb = {"fp64": 8, "fp32": 4, "mixed": 2}[args.precision]
        pbytes = args.d * args.P * args.n_lag * eb + 4 * args.d * args.P * 8
        dps = ms_ps / n_ps * 1e-3
        psrf = {"kernel": "k_psrf_acc (fold of a merged window into the per-chain PSRF accumulators)",
                "bound": "hbm", "achieved": pbytes / dps / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": pbytes / dps / HBM_PEAK, "bytes_per_window": pbytes, "us_per_window": dps * 1e6,
                "worst_sqrt_r_minus_1": res["psrf_worst"]}

    out = {
        "metric": METRIC,
        "value": res["chain_steps_per_s"],
        "unit": "chain-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_window"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "bf16+f16+f64", "fp32": "f32+f64", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"Gaussian target d={args.d} (lambda_i=i^-2, seed 2), P={args.P} chains, "
                               f"n_lag={args.n_lag}, beta={args.beta}, warm start; step = one window",
                   "precision": args.precision, "d": args.d, "P": args.P, "n_lag": args.n_lag},
        "ess_per_s": res["ess_per_s"],
        "steps_per_s": res["steps_per_s"],
        "acceptance": res["acceptance"],
        "stage_ms_per_window": stages,
        "roofline": roofline,
        "psrf": psrf,
        "stopping": res["stopping"],
        "moments": res["moments"],
        "moments_fixed_proposal": res["moments_fixed_proposal"],
    }
    if ref is not None:
        out["fp64"] = {"chain_steps_per_s": ref["chain_steps_per_s"], "ess_per_s": ref["ess_per_s"],
                       "ms_per_window": ref["ms_per_window"], "acceptance": ref["acceptance"],
                       "moments": ref["moments"], "moments_fixed_proposal": ref["moments_fixed_proposal"],
                       "stage_ms_per_window": {k: v[0] / args.profile_windows for k, v in ref["profile"].items()
                                               if v[1]}}
        out["speedup_vs_fp64"] = {"chain_steps": res["chain_steps_per_s"] / ref["chain_steps_per_s"],
                                  "ess": res["ess_per_s"] / ref["ess_per_s"]}
    if not args.no_learned:
        out["learned"] = learned_experiment(args, torch, diam)
    if not args.no_batch:
        out["batch"] = batch_experiment(args, torch, diam)
    if not args.no_families:
        out["families"] = families_experiment(args, torch, diam)
    if not args.no_d1024:
        out["d1024"] = precision_experiment(args, torch, diam)
    if not args.no_local_global:
        out["local_global"] = local_global_experiment(args, torch, diam)
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(tgt, args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
