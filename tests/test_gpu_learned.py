"""Learned-part form on the GPU against the FP64 oracle: the logistic-regression
target, the MLP surrogate (forward, gradient, Adam) and two-stage delayed
acceptance.

Tolerances come from the arithmetic of each kernel:
  * logistic target: t = A x in FP32 (x rounded to FP32, any summation order)
    is within (d + 2) u32 sum_i |a_ji x_i| of the exact product; the per-row
    term y t - softplus(t) moves by at most |t error| (its slope lies in
    (-1, 1)) plus 4 u32 (|t| + softplus(t)) of FP32 evaluation; rows are
    summed in FP64.  B(x) = u32 sum_j [(d + 2) |a_j||x| + 4 (|t_j| + softplus(t_j))].
    A decision is a near-tie when |log alpha - log u| < B(x') + B(x).
  * surrogate: the forward pass runs on FP32 MFMA with bf16-rounded weights;
    the oracle is given the same bf16 values, so only FP32 accumulation
    differs, bounded layer by layer with the running absolute sums.
Near-tie decisions cannot be compared; the oracle then takes the GPU's
decision (its uniform is replaced by one that forces it) and the comparison
goes on, so every later step is still checked.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import diam as od
from oracle import ess as oe
from oracle import mlp as om
from oracle import targets as ot
from paper_1506_05741_amd import diam, synth

U32 = 2.0 ** -24
H = diam.MLP_HIDDEN


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def softplus(t):
    return np.maximum(t, 0.0) + np.log1p(np.exp(-np.abs(t)))


def lp_bound(A, X):
    """B(x) per column of X (d x n): bound on |FP32 target - FP64 target|."""
    d = X.shape[0]
    A64 = A.astype(np.float64)
    T = A64 @ X
    S = np.abs(A64) @ np.abs(X)
    return U32 * np.sum((d + 2) * S + 4.0 * (np.abs(T) + softplus(T)), axis=0) + 1e-9


class LogReg:
    def __init__(self, n_obs, d, P, n_lag, seed=5, beta=0.3, surrogate=False, train_max=0, prec="fp64"):
        self.data = synth.logreg_data(n=n_obs, d=d, seed=seed, prior_var=10.0)
        self.d, self.P, self.n_lag = d, P, n_lag
        rng = np.random.default_rng(seed + 1)
        x0 = self.data.w_true[:, None] + 0.1 * rng.standard_normal((d, P))
        self.A, self.y = self.data.A, self.data.y
        self.logpi = lambda X: ot.logreg_logpdf(self.A, self.y, self.data.prior_var, X)
        self.o = od.DiamOracle(self.logpi, d, P, n_lag, beta, X=x0)
        cfg = diam.make_config(d, P, n_lag, prec, beta=beta, seed=77, surrogate=surrogate, train_max=train_max)
        self.s = diam.Sampler(cfg, None, None, dev(x0.T), A=dev(self.A, torch.float32),
                              y=dev(self.y, torch.float32), prior_var=self.data.prior_var)

    def gx(self):
        return host(self.s.get_f64(diam.F_X, (self.P, self.d))).T

    def glp(self):
        return host(self.s.get_f64(diam.F_LOGP, (self.P,)))

    def surrogate(self, X):
        return host(self.s.surrogate_eval(dev(X.T)))


def force(u, acc_gpu, near):
    """Uniforms with which the oracle takes the GPU's decision on near ties."""
    u = u.copy()
    u[near & acc_gpu] = 2.0 ** -60
    u[near & ~acc_gpu] = 1.0
    return u


def step_and_compare(pr, W, u):
    """One plain step on both sides.  Returns the number of forced near ties."""
    o, P = pr.o, pr.P
    Xp = od.diam_proposal(o.X, o.x_ref, o.A, W.T, o.beta, o.alpha)
    Zp = od.whiten(o.A, o.x_ref, Xp)
    la_o = od.log_accept_ratio(pr.logpi(Xp), o.lp, Zp, o.Z, o.alpha)
    tie = lp_bound(pr.A, Xp) + lp_bound(pr.A, o.X)
    pr.s.step_batch(1, dev(W[None]), dev(u[None]))
    la_g = host(pr.s.get_f64(diam.F_LA, (P,)))
    acc_g = host(pr.s.get(diam.F_ACC)).astype(bool)
    near = np.abs(la_o - np.log(u)) < tie
    far = ~near
    assert np.array_equal(acc_g[far], (np.log(u) < la_o)[far]), np.nonzero(acc_g[far] != (np.log(u) < la_o)[far])
    assert np.all(np.abs(la_g - la_o) <= tie), np.max(np.abs(la_g - la_o) / tie)
    # a forced decision at a genuine tie: the oracle's la sits within the
    # bound of log u, so the forcing uniforms cannot contradict it
    assert not np.any(near & ~acc_g & (la_o > 0.0))
    acc_o, _ = o.step(W.T, force(u, acc_g, near))
    assert np.array_equal(acc_o, acc_g)
    return int(near.sum())


def check_states(pr, tol):
    Xg = pr.gx()
    err = np.linalg.norm(Xg - pr.o.X, axis=0) / np.linalg.norm(pr.o.X, axis=0)
    assert err.max() <= tol, err.max()
    lp = pr.glp()
    lp_ref = pr.logpi(Xg)
    assert np.all(np.abs(lp - lp_ref) <= lp_bound(pr.A, Xg)), np.max(np.abs(lp - lp_ref) / lp_bound(pr.A, Xg))


def test_logistic_target_against_fp64_definition():
    # 1000 observations: 15 full 64-row blocks and a ragged 40; d = 40 is a
    # ragged K; 70 chains span two column tiles
    pr = LogReg(1000, 40, 70, 10)
    X = pr.gx()
    lp = pr.glp()
    lp_ref = pr.logpi(X)
    err = np.abs(lp - lp_ref)
    B = lp_bound(pr.A, X)
    log(f"logistic log pi: max |err| {err.max():.3e}, max err / bound {np.max(err / B):.3e}")
    assert np.all(err <= B)
    assert np.allclose(lp_ref, pr.o.lp, rtol=0, atol=0)


def test_logistic_decision_parity():
    d, P, n_lag, windows = 40, 70, 20, 3
    pr = LogReg(1000, d, P, n_lag)
    W = synth.draw_normals(d, P, windows * n_lag, 21)
    U = synth.draw_uniforms(P, windows * n_lag, 22)
    forced = 0
    for k in range(windows):
        for t in range(k * n_lag, (k + 1) * n_lag):
            forced += step_and_compare(pr, W[t], U[t])
        kappa = np.linalg.cond(pr.o.A) ** 2
        check_states(pr, max(1e-12, kappa * np.finfo(float).eps))
        pr.s.merge_moments()
        pr.o.merge_moments()
        S = host(pr.s.get_f64(diam.F_S, (d, d))).T
        assert np.linalg.norm(S - pr.o.S_glob) <= 1e-12 * np.linalg.norm(pr.o.S_glob)
        st, j = pr.s.update_proposal()
        assert st == diam.OK and pr.o.update_proposal() == od.OK and j == pr.o.last_jitter
        log(f"  window {k}: accepted {int(pr.o.n_accepted.sum())}, forced near ties so far {forced}")
    assert int(pr.o.n_accepted.sum()) > 0.2 * P * n_lag * windows


def _gpu_params(s, d):
    p = host(s.get(diam.F_MLP_PARAMS).view(torch.float32)).astype(np.float64)
    sizes = [H * d, H, H * H, H, H, 1]
    shapes = [(H, d), (H,), (H, H), (H,), (1, H), (1,)]
    out, o = [], 0
    for n, sh in zip(sizes, shapes):
        out.append(p[o:o + n].reshape(sh))
        o += n
    assert o == p.size
    return out


def _gpu_stats(s, d):
    st = host(s.get(diam.F_MLP_STATS).view(torch.float32)).astype(np.float64)
    return st[:d], st[d:2 * d], st[2 * d], st[2 * d + 1]


def _training_pairs(n, d, seed):
    data = synth.logreg_data(n=1000, d=d, seed=5, prior_var=10.0)
    rng = np.random.default_rng(seed)
    X = data.w_true[:, None] + 0.2 * rng.standard_normal((d, n))
    lp = ot.logreg_logpdf(data.A, data.y, data.prior_var, X)
    return X, lp


def _standardise_f32(X, mean, scale):
    """The kernel's standardisation: FP32 x, FP32 (x - mean) * scale."""
    xf = X.astype(np.float32)
    return ((xf - mean.astype(np.float32)[:, None]) * scale.astype(np.float32)[:, None]).astype(np.float64)


def _grad_bound(params, Xs, t):
    """First-order bound of the FP32 backward pass's deviation from FP64 at the
    same bf16 weights: each contraction of length K is within (K + 2) u32 of
    the sum of |terms|, carried through the layers with |gelu'| <= 1.13."""
    W1, b1, W2, b2, W3, b3 = [np.abs(p) for p in params]
    out, (xs, a1, h1, a2, h2) = om.forward(params, Xs)
    n = out.size
    D = Xs.shape[0]
    g = 1.13
    e_a1 = (D + 2) * U32 * (W1 @ np.abs(xs) + b1[:, None])
    e_h1 = g * e_a1 + U32 * np.abs(h1)
    e_a2 = W2 @ e_h1 + (H + 2) * U32 * (W2 @ np.abs(h1) + b2[:, None])
    e_h2 = g * e_a2 + U32 * np.abs(h2)
    e_out = (W3 @ e_h2 + (H + 2) * U32 * (W3 @ np.abs(h2)))[0]
    r = np.abs(out - t) + e_out
    e_g = (2.0 / n) * (e_out + U32 * r)
    # gradient of W3 and the back-propagated signals, same pattern
    gW3 = (2.0 / n) * r @ np.abs(h2).T
    eW3 = e_g @ np.abs(h2).T + (2.0 / n) * r @ e_h2.T + (n + 2) * U32 * gW3
    return eW3, e_g


def test_surrogate_gradient_and_adam_step_against_oracle():
    d, P, n = 40, 70, 3000
    pr = LogReg(1000, d, P, 10, surrogate=True, train_max=n)
    X, lp = _training_pairs(n, d, 31)
    Xd, lpd = dev(X.T), dev(lp)
    pr.s.surrogate_train(Xd, lpd, steps=0, batch=200, lr=1e-3, seed=5)
    p0 = _gpu_params(pr.s, d)
    mean, scale, omean, ostd = _gpu_stats(pr.s, d)
    assert np.allclose(mean, X.mean(axis=1), rtol=1e-6, atol=1e-6)
    assert np.allclose(1.0 / scale, X.std(axis=1), rtol=1e-5)
    assert abs(omean - lp.mean()) <= 1e-6 * abs(lp.mean()) and abs(ostd - lp.std()) <= 1e-5 * lp.std()
    # He init: N(0, 2 / fan_in) weights, zero biases
    assert np.all(p0[1] == 0) and np.all(p0[3] == 0) and np.all(p0[5] == 0)
    assert abs(p0[0].std() * math.sqrt(d / 2.0) - 1.0) < 0.02
    assert abs(p0[2].std() * math.sqrt(H / 2.0) - 1.0) < 0.02

    loss = pr.s.surrogate_train(Xd, lpd, steps=1, batch=200, lr=1e-3, seed=5)
    g_gpu = host(pr.s.get(diam.F_MLP_GRAD).view(torch.float32)).astype(np.float64)
    idx = host(pr.s.get(diam.F_MLP_BATCH).view(torch.int32))
    assert idx.shape == (200,) and idx.min() >= 0 and idx.max() < n
    p1 = _gpu_params(pr.s, d)
    eff = [om.round_bf16(p) for p in p0]
    W3 = eff[4]
    params = [eff[0], eff[1], eff[2], eff[3], W3, eff[5]]
    Xs = _standardise_f32(X[:, idx], mean, scale)
    # the kernel standardises the targets with FP64 statistics, then rounds to FP32
    m64 = lp.mean()
    s64 = math.sqrt(max(np.mean(lp * lp) - m64 * m64, 0.0))
    t = ((lp[idx] - m64) / s64).astype(np.float32).astype(np.float64)
    loss_o, grads = om.loss_and_grad(params, Xs, t)
    g_o = np.concatenate([g.ravel() for g in grads])
    assert g_o.size == g_gpu.size
    rel = np.linalg.norm(g_gpu - g_o) / np.linalg.norm(g_o)
    eW3, _ = _grad_bound(params, Xs, t)
    gw3_err = np.abs(g_gpu[-H - 1:-1] - grads[4].ravel())
    log(f"surrogate gradient: relative error {rel:.3e}, W3 block max err / bound "
        f"{np.max(gw3_err / eW3.ravel()):.3e}; loss {loss:.4f} vs {loss_o:.4f}")
    assert np.all(gw3_err <= eW3.ravel())
    assert rel < 1e-4
    assert abs(loss - loss_o) <= 1e-5 * max(1.0, loss_o)
    # one Adam step from zero moments, on the GPU's gradient
    cuts = np.cumsum([q.size for q in p0])[:-1]
    g_blocks = [g.reshape(q.shape) for g, q in zip(np.split(g_gpu, cuts), p0)]
    zeros = [np.zeros_like(q) for q in p0]
    new, _, _ = om.adam_step(p0, g_blocks, zeros, zeros, 1, lr=1e-3)
    for a, b in zip(p1, new):
        assert np.allclose(a, b, rtol=1e-6, atol=1e-9)


def _forward_bound(params, Xs):
    W1, b1, W2, b2, W3, b3 = [np.abs(p) for p in params]
    out, (xs, a1, h1, a2, h2) = om.forward(params, Xs)
    D = Xs.shape[0]
    e_xs = U32 * np.abs(xs) * 3
    e_a1 = (D + 2) * U32 * (W1 @ np.abs(xs) + b1[:, None]) + W1 @ e_xs
    e_h1 = 1.13 * e_a1 + U32 * np.abs(h1) * 2
    e_a2 = W2 @ e_h1 + (H + 2) * U32 * (W2 @ np.abs(h1) + b2[:, None])
    e_h2 = 1.13 * e_a2 + U32 * np.abs(h2) * 2
    return out, (W3 @ e_h2 + (H + 2) * U32 * (W3 @ np.abs(h2)))[0]


def test_surrogate_forward_against_oracle():
    d, P, n = 40, 70, 3000
    pr = LogReg(1000, d, P, 10, surrogate=True, train_max=n)
    X, lp = _training_pairs(n, d, 41)
    loss = pr.s.surrogate_train(dev(X.T), dev(lp), steps=300, batch=256, lr=1e-3, seed=9)
    params = [om.round_bf16(p) for p in _gpu_params(pr.s, d)]
    mean, scale, omean, ostd = _gpu_stats(pr.s, d)
    Xq, lpq = _training_pairs(300, d, 43)
    s_gpu = host(pr.s.surrogate_eval(dev(Xq.T)))
    out, e_out = _forward_bound(params, _standardise_f32(Xq, mean, scale))
    s_o = out * ostd + omean
    err = np.abs(s_gpu - s_o)
    bound = e_out * ostd + U32 * (np.abs(out) * ostd + abs(omean)) * 2
    log(f"surrogate forward: loss {loss:.4f}, max err {err.max():.3e}, max err / bound {np.max(err / bound):.3e}; "
        f"held-out corr {np.corrcoef(s_gpu, lpq)[0, 1]:.4f}")
    assert np.all(err <= bound)
    assert loss < 0.1
    assert np.corrcoef(s_gpu, lpq)[0, 1] > 0.85


@pytest.mark.parametrize("form", [1, 2])
def test_delayed_acceptance_parity(form):
    """Two-stage delayed acceptance against the oracle's step_delayed, in both
    surrogate forms (1: s = r, the network; 2: s = r - |z|^2 / (2 alpha^2)).
    The surrogate is an input of the acceptance rule: the oracle evaluates the
    GPU-trained network through diam_surrogate_eval (its arithmetic is
    checked against the FP64 oracle network above)."""
    d, P, n_lag = 40, 70, 20
    pr = LogReg(1000, d, P, n_lag, surrogate=form, train_max=4000, beta=0.6)
    o = pr.o
    W = synth.draw_normals(d, P, 3 * n_lag, 51)
    U = synth.draw_uniforms(P, n_lag, 52)
    Xs, lps = [], []
    for t in range(n_lag):                                    # one window of plain steps, pairs collected
        step_and_compare(pr, W[t], U[t])
        Xs.append(pr.gx())
        lps.append(pr.glp())

    def merge_update():
        pr.s.merge_moments()
        o.merge_moments()
        S = host(pr.s.get_f64(diam.F_S, (d, d))).T
        assert np.linalg.norm(S - o.S_glob) <= 1e-12 * np.linalg.norm(o.S_glob)
        assert pr.s.update_proposal()[0] == diam.OK and o.update_proposal() == od.OK

    merge_update()
    X = np.concatenate(Xs, axis=1)
    pr.s.surrogate_train(dev(X.T), dev(np.concatenate(lps)), steps=300, batch=256, lr=1e-3, seed=3)
    pr.s.set_delayed_acceptance(True)

    def surrogate(Xq):
        r = pr.surrogate(Xq)
        if form == 2:
            Zq = od.whiten(o.A, o.x_ref, Xq)
            r = r - np.sum(Zq * Zq, axis=0) / (2.0 * o.alpha ** 2)
        return r

    r_cur = pr.surrogate(o.X)
    assert np.allclose(host(pr.s.get_f64(diam.F_SURR, (P,))), r_cur, rtol=1e-6, atol=1e-6)
    U2 = synth.draw_uniforms(P, 2 * n_lag, 53, stages=2)
    npass_prev = host(pr.s.get(diam.F_NPASS).view(torch.int32)).copy()
    forced = survivors = accepted = 0
    for k in range(2 * n_lag):
        if k == n_lag:
            merge_update()
        s_cur = surrogate(o.X)
        w = W[n_lag + k]
        u1, u2 = U2[k, 0], U2[k, 1]
        Xp = od.diam_proposal(o.X, o.x_ref, o.A, w.T, o.beta, o.alpha)
        Zp = od.whiten(o.A, o.x_ref, Xp)
        sp = surrogate(Xp)
        la1 = od.log_accept_ratio(sp, s_cur, Zp, o.Z, o.alpha)
        la2 = (pr.logpi(Xp) - o.lp) - (sp - s_cur)
        tie2 = lp_bound(pr.A, Xp) + lp_bound(pr.A, o.X)
        pr.s.step_batch(1, dev(w[None]), dev(U2[k:k + 1]))
        acc_g = host(pr.s.get(diam.F_ACC)).astype(bool)
        la_g = host(pr.s.get_f64(diam.F_LA, (P,)))
        npass = host(pr.s.get(diam.F_NPASS).view(torch.int32)).copy()
        pass_g = (npass - npass_prev).astype(bool)
        npass_prev = npass
        near1 = np.abs(la1 - np.log(u1)) < 1e-9
        assert np.array_equal(pass_g[~near1], (np.log(u1) < la1)[~near1])
        near2 = pass_g & (np.abs(la2 - np.log(u2)) < tie2)
        far2 = pass_g & ~near2
        assert np.array_equal(acc_g[far2], (np.log(u2) < la2)[far2])
        assert np.all(np.abs(la_g[pass_g] - la2[pass_g]) <= tie2[pass_g])
        assert np.all(np.isneginf(la_g[~pass_g])) and not np.any(acc_g[~pass_g])
        acc_o, pass_o, _ = o.step_delayed(w.T, force(u1, pass_g, near1), force(u2, acc_g, near2), surrogate, s_cur)
        assert np.array_equal(pass_o, pass_g) and np.array_equal(acc_o, acc_g)
        forced += int(near1.sum() + near2.sum())
        survivors += int(pass_g.sum())
        accepted += int(acc_g.sum())
    check_states(pr, max(1e-12, np.linalg.cond(o.A) ** 2 * np.finfo(float).eps))
    assert np.allclose(host(pr.s.get_f64(diam.F_SURR, (P,))), pr.surrogate(o.X), rtol=1e-6, atol=1e-6)
    log(f"delayed acceptance (form {form}): {survivors} stage-1 survivors, {accepted} accepted of {2 * n_lag * P}, "
        f"{forced} forced near ties")
    assert 0 < survivors < 2 * n_lag * P and accepted > 0
    merge_update()


def test_learned_form_state_errors():
    pr = LogReg(1000, 40, 8, 10)
    with pytest.raises(diam.DiamError) as e:
        pr.s.set_delayed_acceptance(True)
    assert e.value.status == diam.E_STATE
    pr2 = LogReg(1000, 40, 8, 10, surrogate=True, train_max=100)
    with pytest.raises(diam.DiamError) as e:
        pr2.s.set_delayed_acceptance(True)              # not trained
    assert e.value.status == diam.E_STATE
    X, lp = _training_pairs(200, 40, 1)
    with pytest.raises(diam.DiamError) as e:            # more pairs than reserved
        pr2.s.surrogate_train(dev(X.T), dev(lp), steps=1)
    assert e.value.status == diam.E_ARG


def _run_logistic(data, mode, C, P, n_lag, beta, windows, use_da, n_pairs=4096, train_steps=1500):
    """Warm-started sampler on the logistic posterior; `windows` traced
    windows after a collection phase of n_pairs states (which, with use_da,
    train the surrogate before delayed acceptance is switched on).  Returns
    the traces (steps x 3 x P: log pi, v_max^T x, v_min^T x), the seconds of
    the traced windows, the accepted count and the stage-1 survivors."""
    import time
    d = data.A.shape[1]
    rng = np.random.default_rng(17)
    x0 = mode[:, None] + np.linalg.cholesky(C) @ rng.standard_normal((d, P))
    cfg = diam.make_config(d, P, n_lag, "fp32", beta=beta, seed=91, surrogate=2 if use_da else 0,
                           train_max=n_pairs)
    s = diam.Sampler(cfg, None, None, dev(x0.T), A=dev(data.A, torch.float32), y=dev(data.y, torch.float32),
                     prior_var=data.prior_var)
    assert s.seed_moments(dev(C + np.outer(mode, mode)), dev(mode), 10 * P * n_lag)[0] == diam.OK
    collect = -(-n_pairs // P)
    Xtr = torch.empty((collect * P, d), dtype=torch.float64, device="cuda")
    ltr = torch.empty(collect * P, dtype=torch.float64, device="cuda")
    for k in range(collect):                                  # identical in both runs
        s.step_batch(1)
        Xtr[k * P:(k + 1) * P] = s.get_f64(diam.F_X, (P, d))
        ltr[k * P:(k + 1) * P] = s.get_f64(diam.F_LOGP, (P,))
        if s.stats()["steps_in_window"] == n_lag:
            s.merge_moments()
            assert s.update_proposal()[0] == diam.OK
    rest = n_lag - s.stats()["steps_in_window"]
    if rest < n_lag:
        s.step_batch(rest)
        s.merge_moments()
        assert s.update_proposal()[0] == diam.OK
    loss = None
    if use_da:
        loss = s.surrogate_train(Xtr[:n_pairs], ltr[:n_pairs], steps=train_steps, batch=256, lr=1e-3, seed=5)
        s.set_delayed_acceptance(True)
    ev, V = np.linalg.eigh(C)
    proj = dev(np.stack([V[:, -1], V[:, 0]]))
    trace = torch.empty((windows * n_lag, 3, P), dtype=torch.float64, device="cuda")
    s.set_trace(proj, trace)
    nacc0 = int(s.get(diam.F_NACC).view(torch.int32).sum())
    npass0 = int(s.get(diam.F_NPASS).view(torch.int32).sum()) if use_da else 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(windows):
        s.step_batch(n_lag)
        s.merge_moments()
        assert s.update_proposal()[0] == diam.OK
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    nacc = int(s.get(diam.F_NACC).view(torch.int32).sum()) - nacc0
    npass = (int(s.get(diam.F_NPASS).view(torch.int32).sum()) - npass0) if use_da else windows * n_lag * P
    tr = host(trace)
    s.close()
    return tr, T, nacc, npass, loss


def test_delayed_acceptance_matches_plain_posterior_and_reports_gain():
    """Delayed acceptance with the trained surrogate against the plain
    sampler on the same logistic-regression posterior (n = 20000, d = 64,
    P = 128, beta = 1, Laplace warm start): the posterior mean of log pi, the
    means and variances of v_max^T x and v_min^T x agree within 4 combined
    Monte Carlo standard errors (the plain FP32 sampler is the judge).  The
    test also measures what the network gains: the share of exact target
    evaluations stage 1 saves, the ESS per exact evaluation and the ESS per
    second of delayed acceptance relative to the plain sampler."""
    n, d, P, n_lag, windows = 20000, 64, 128, 100, 30
    data = synth.logreg_data(n=n, d=d, seed=4)
    mode, C = synth.logreg_laplace(data)
    res = {}
    for use_da in (False, True):
        res[use_da] = _run_logistic(data, mode, C, P, n_lag, 1.0, windows, use_da)
    worst = 0.0
    report = []
    ess = {}
    for use_da in (False, True):
        tr = res[use_da][0]
        ess[use_da] = min(oe.ess_chains(tr[:, f, :]) for f in range(3))
    for f, name in enumerate(("log pi", "v_max^T x", "v_min^T x")):
        stats = []
        for use_da in (False, True):
            x = res[use_da][0][:, f, :]
            sq = (x - x.mean()) ** 2
            stats.append(((x.mean(), x.std() / math.sqrt(oe.ess_chains(x))),
                          (sq.mean(), sq.std() / math.sqrt(oe.ess_chains(sq)))))
        for k in ((0,) if f == 0 else (0, 1)):
            (a, sa), (b, sb) = stats[0][k], stats[1][k]
            z = (b - a) / math.sqrt(sa * sa + sb * sb)
            worst = max(worst, abs(z))
            report.append(f"{name} {'mean' if k == 0 else 'variance'} z {z:+.2f}")
    steps = windows * n_lag * P
    plain, da = res[False], res[True]
    saved = 1.0 - da[3] / steps
    per_eval = (ess[True] / da[3]) / (ess[False] / plain[3])
    per_s = (ess[True] / da[1]) / (ess[False] / plain[1])
    log(f"delayed acceptance vs plain (logistic n={n}, d={d}, P={P}, beta=1): " + ", ".join(report)
        + f"; acceptance plain {plain[2] / steps:.3f}, DA {da[2] / steps:.3f}, stage-1 pass {da[3] / steps:.3f}; "
          f"surrogate loss {da[4]:.4f}; the network saves {100 * saved:.1f} % of exact evaluations, "
          f"ESS per exact evaluation x{per_eval:.2f}, ESS/s x{per_s:.2f} of the plain sampler")
    assert worst < 4.0
    assert 0.0 < saved < 1.0                                  # stage 1 screens some proposals, not all
    assert da[2] > 0.2 * steps
