"""Batched form on the GPU: G independent Gaussian problems in grouped launches.

* Against separate samplers: each problem of the batch, fed through a plain
  DIAM_FP32 sampler with the batch's own normals and uniforms, gives bitwise
  the same states, log densities, accept decisions, moments, pivot and factor
  (the grouped launches run the single-problem tile bodies; the default
  target tile keeps the accumulation order).  Dimensions are ragged (1, 40,
  70, 128, 200): partial tiles, several Cholesky blocks and a degenerate d = 1.
* Graph replays against eager launches, with unrelated eager work between
  the replays, bitwise on every window.
* With the autotuned tile shape the chains of every problem reproduce its
  posterior moments within 4 Monte Carlo standard errors.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ess as oe
from paper_1506_05741_amd import diam, synth


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def problems(dims, P, seed0):
    ts = [synth.gaussian_target(int(d), seed0 + g) for g, d in enumerate(dims)]
    x0 = [synth.gaussian_exact_draws(t, P, seed0 + 100 + g) for g, t in enumerate(ts)]
    return ts, x0


def make_batch(ts, x0, P, n_lag, seed, N0):
    cfg = diam.make_batch_config(len(ts), P, n_lag, beta=0.3, seed=seed)
    b = diam.Batch(cfg, [dev(t.mu) for t in ts], [dev(t.R, torch.float32) for t in ts], [dev(x.T) for x in x0])
    S = [dev(synth.gaussian_warm_moments(t)[0]) for t in ts]
    m = [dev(synth.gaussian_warm_moments(t)[1]) for t in ts]
    st, j = b.seed_moments(S, m, N0)
    assert st == diam.OK
    return b, j


FIELDS = [diam.F_X, diam.F_Z, diam.F_LOGP, diam.F_ZQ, diam.F_XREF, diam.F_L, diam.F_S, diam.F_M, diam.F_NACC]


def test_batch_matches_separate_samplers():
    dims, P, n_lag, windows = [40, 128, 1, 200, 70], 32, 8, 3
    ts, x0 = problems(dims, P, 11)
    N0 = 10 * P * n_lag
    b, jb = make_batch(ts, x0, P, n_lag, 5, N0)
    singles = []
    for t, x in zip(ts, x0):
        cfg = diam.make_config(t.d, P, n_lag, "fp32", beta=0.3, seed=9)
        s = diam.Sampler(cfg, dev(t.mu), dev(t.R, torch.float32), dev(x.T))
        S0, m0 = synth.gaussian_warm_moments(t)
        st, j = s.seed_moments(dev(S0), dev(m0), N0)
        assert st == diam.OK
        singles.append(s)
    for f in FIELDS:
        for g in range(len(dims)):
            assert torch.equal(b.get(g, f), singles[g].get(f)), (f, g)
    for w in range(windows):
        st, jit = b.window()
        assert st == diam.OK
        for g, (t, s) in enumerate(zip(ts, singles)):
            ld = (t.d + 3) // 4 * 4                         # the batch keeps normals in rows padded to 4
            W = b.get(g, diam.F_W).view(torch.float32).reshape(n_lag, P, ld)[:, :, : t.d].double().contiguous()
            U = b.get(g, diam.F_U).view(torch.float64).reshape(n_lag, P).contiguous()
            s.step_batch(n_lag, W, U)
            assert torch.equal(b.get(g, diam.F_ACC), s.get(diam.F_ACC)), (w, g)
            assert torch.equal(b.get(g, diam.F_LA), s.get(diam.F_LA)), (w, g)
            s.merge_moments()
            st, j = s.update_proposal()
            assert st == diam.OK and j == jit[g]
            for f in FIELDS:
                assert torch.equal(b.get(g, f), s.get(f)), (w, g, f)
        acc = sum(int(s.get(diam.F_NACC).view(torch.int32).sum()) for s in singles)
        log(f"window {w}: all {len(dims)} problems bitwise equal to separate samplers; accepted so far {acc}")
    assert b.stats()["windows"] == windows


def test_graph_replays_match_eager_windows():
    dims, P, n_lag = [33, 96, 150], 32, 16
    ts, x0 = problems(dims, P, 21)
    bg, _ = make_batch(ts, x0, P, n_lag, 3, 10 * P * n_lag)
    be, _ = make_batch(ts, x0, P, n_lag, 3, 10 * P * n_lag)
    be.set_graph(False)
    a = torch.randn(512, 512, device="cuda")
    for w in range(4):
        assert bg.window()[0] == diam.OK
        _ = (a @ a).sum().item()                      # unrelated eager work between replays
        assert be.window()[0] == diam.OK
        torch.cuda.synchronize()
        for g in range(len(dims)):
            for f in FIELDS + [diam.F_W, diam.F_U, diam.F_ACC]:
                assert torch.equal(bg.get(g, f), be.get(g, f)), (w, g, f)
    log("graph replays equal eager windows bitwise over 4 windows")


def _worst_z(t, X):
    n, d, P = X.shape
    V = np.concatenate([np.eye(d)[:, : min(d, 8)], t.Q[:, [0, -1]], synth.unit_vectors(d, 8, 5)], axis=1)
    worst = 0.0
    for j in range(V.shape[1]):
        v = V[:, j]
        f = np.einsum("i,nip->np", v, X)
        for g, truth in ((f, v @ t.mu), ((f - v @ t.mu) ** 2, v @ t.Sigma @ v)):
            ess = oe.ess_chains(g)
            worst = max(worst, abs(g.mean() - truth) / (g.std() / math.sqrt(ess)))
    return worst


def test_autotuned_batch_reproduces_posterior_moments():
    dims, P, n_lag, windows = [24, 48, 96], 32, 64, 40
    ts, x0 = problems(dims, P, 31)
    b, _ = make_batch(ts, x0, P, n_lag, 8, 10 * P * n_lag)
    choice, us = b.autotune(reps=10)
    log(f"autotune: choice {diam.BATCH_TILES[choice]}, us per launch {us}")
    assert 0 <= choice < len(diam.BATCH_TILES) and all(v > 0 for v in us.values())
    assert us[diam.BATCH_TILES[choice]] == min(us.values())
    ends = [[] for _ in dims]
    for _ in range(windows):
        assert b.window()[0] == diam.OK
        for g, d in enumerate(dims):
            ends[g].append(host(b.get_f64(g, diam.F_X, (P, d))).T)
    for g, t in enumerate(ts):
        worst = _worst_z(t, np.stack(ends[g]))
        acc = host(b.get(g, diam.F_NACC).view(torch.int32)).sum() / (P * n_lag * windows)
        log(f"problem {g} (d={t.d}): worst |z| {worst:.2f}, acceptance {acc:.3f}")
        assert worst < 4.0 and acc > 0.5
