"""Degenerate and ragged sizes of the widened parts of the path against the
oracle, FP64:

* local-global logistics (M = 2) with one chain in one dimension, and with a
  ragged d = 65 (two 64-row tiles, the second one row deep);
* AM, pCN and RW with one chain in one dimension;
* PSRF with the fewest chains it accepts (P = 2) in one dimension;
* a twisted target of odd dimension (d = 41: twisted rows 1 and 3, the last
  row unpaired), and per-chain factors (M = 2) on a twisted target.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import diam as od
from oracle import psrf as op
from oracle import targets as ot
from paper_1506_05741_amd import diam, synth
from tests.gpu_parity import assert_few_forced, oracle_follow


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def run_parity(s, o, d, P, n_lag, windows, seed, adopt_shared, tie=1e-9):
    """Windows of decision parity (the oracle following the GPU through
    near-ties); after each update the oracle takes the GPU's factors
    (independent FP64 roundings).  Returns the accepted count."""
    rng = np.random.default_rng(seed)
    total = forced = 0
    for k in range(windows):
        W = rng.standard_normal((n_lag, P, d))
        U = synth.draw_uniforms(P, n_lag, 300 + k + 17 * seed)
        s.step_batch(n_lag, dev(W), dev(U))
        acc_g = host(s.get(diam.F_ACC)).reshape(n_lag, P).astype(bool)
        la_g = host(s.get_f64(diam.F_LA, (n_lag, P)))
        a, f = oracle_follow(o, W, U, acc_g, la_g, tie, where=f"d={d} P={P} window {k}")
        total, forced = total + a, forced + f
        assert rel(host(s.get_f64(diam.F_X, (P, d))).T, o.X) <= 1e-12, k
        s.merge_moments()
        o.merge_moments()
        st, j = s.update_proposal()
        assert st == diam.OK and o.update_proposal() == od.OK and j == o.last_jitter
        if getattr(o, "Ap", None) is not None:
            Lp = host(s.get_f64(diam.F_LP, (P, d, d))).transpose(0, 2, 1)
            assert rel(Lp, o.Ap) <= 1e-10 and rel(host(s.get_f64(diam.F_XREFP, (P, d))).T, o.xrp) <= 1e-12
            o.Ap = Lp.copy()
            for p in range(P):
                o.Z[:, p:p + 1] = od.whiten(o.Ap[p], o.xrp[:, p], o.X[:, p:p + 1])
        elif adopt_shared:
            L = host(s.get_f64(diam.F_L, (d, d))).T
            assert rel(L, o.A) <= 1e-10
            o.A = L.copy()
            o.Z = od.whiten(o.A, o.x_ref, o.X)
    print(f"\n  compared {windows} windows of {n_lag} steps x {P} chains, each merged and updated; "
          f"{forced} forced near-ties", flush=True)
    assert_few_forced(forced, windows * n_lag * P)
    return total


@pytest.mark.parametrize("d,P", [(1, 1), (65, 3)])
def test_local_global_degenerate_and_ragged(d, P):
    n_lag, M = 3 if d == 1 else 8, 2
    t = synth.gaussian_target(d, 3)
    x0 = synth.gaussian_exact_draws(t, P, 4)
    s = diam.Sampler(diam.make_config(d, P, n_lag, "fp64", beta=0.5, seed=2, M=M), dev(t.mu), dev(t.R), dev(x0.T))
    o = od.DiamOracle(lambda X: ot.gaussian_logpdf(t.R, t.mu, X), d, P, n_lag, 0.5, X=x0, M=M)
    S0, m0 = synth.gaussian_warm_moments(t)
    assert s.seed_moments(dev(S0), dev(m0), 3 * P * n_lag)[0] == diam.OK
    assert o.seed_moments(S0, m0, 3 * P * n_lag) == od.OK
    o.A = host(s.get_f64(diam.F_L, (d, d))).T.copy()
    o.Z = od.whiten(o.A, o.x_ref, o.X)
    total = run_parity(s, o, d, P, n_lag, 5, 1, adopt_shared=True)
    print(f"\n[M=2 d={d} P={P}] parity, {total} accepted", flush=True)
    assert total > 0


@pytest.mark.parametrize("prop", ["am", "pcn", "rw"])
def test_families_one_chain_one_dimension(prop):
    d, P, n_lag = 1, 1, 6
    t = synth.paper_gaussian("pi2", 10, 5)                 # take its first coordinate's scale
    mu, R = np.zeros(1), np.array([[1.0 / np.sqrt(t.lam[0])]])
    x0 = np.array([[0.3]])
    s = diam.Sampler(diam.make_config(d, P, n_lag, "fp64", beta=0.5, seed=4, proposal=prop), dev(mu), dev(R), dev(x0.T))
    o = od.DiamOracle(lambda X: ot.gaussian_logpdf(R, mu, X), d, P, n_lag, 0.5, X=x0, proposal=prop)
    if prop == "am":
        S = np.array([[t.lam[0]]])
        assert s.seed_moments(dev(S), dev(mu), 20)[0] == diam.OK
        assert o.seed_moments(S, mu, 20) == od.OK
        o.A = host(s.get_f64(diam.F_L, (1, 1))).T.copy()
        o.Z = od.whiten(o.A, o.x_ref, o.X)
    total = run_parity(s, o, d, P, n_lag, 4, 2, adopt_shared=(prop == "am"))
    print(f"\n[{prop} d=1 P=1] parity, {total} accepted", flush=True)
    assert total > 0


def test_psrf_two_chains_one_dimension():
    d, P, n_lag = 1, 2, 5
    mu, R = np.array([0.5]), np.array([[2.0]])
    x0 = np.array([[0.1, 0.9]])
    s = diam.Sampler(diam.make_config(d, P, n_lag, "fp64", beta=0.6, seed=6), dev(mu), dev(R), dev(x0.T))
    assert s.seed_moments(dev(np.array([[0.25 + 0.25]])), dev(mu), 10)[0] == diam.OK
    s.psrf_enable(True)
    chains = []
    for _ in range(3):
        for _ in range(n_lag):
            s.step_batch(1)
            chains.append(host(s.get_f64(diam.F_X, (P, d))))
        s.merge_moments()
        assert s.update_proposal()[0] == diam.OK
    ref = op.psrf(np.stack(chains, axis=1))
    got, worst = s.psrf()
    assert np.max(np.abs(host(got) - ref)) < 1e-11      # states folded as pivot + stored shift
    assert worst == pytest.approx(float(ref[0] - 1.0), abs=1e-11)


def test_twisted_target_odd_dimension():
    d, P, n_lag = 41, 4, 8
    t = synth.twisted_target(d, 2, 2.0)
    assert list(np.nonzero(t.c)[0]) == [1, 3]
    x0 = synth.twisted_exact_draws(t, P, 3)
    s = diam.Sampler(diam.make_config(d, P, n_lag, "fp64", beta=0.3, alpha=1.3, seed=7), dev(t.mu), dev(t.R),
                     dev(x0.T), twist=dev(t.c))
    o = od.DiamOracle(lambda X: ot.twisted_logpdf(t.R, t.mu, t.c, X), d, P, n_lag, 0.3, alpha=1.3, X=x0)
    np.testing.assert_allclose(host(s.get_f64(diam.F_LOGP, (P,))), o.lp, rtol=1e-12, atol=1e-12)
    S0, m0 = synth.twisted_warm_moments(t)
    assert s.seed_moments(dev(S0), dev(m0), 10 * P * n_lag)[0] == diam.OK
    assert o.seed_moments(S0, m0, 10 * P * n_lag) == od.OK
    o.A = host(s.get_f64(diam.F_L, (d, d))).T.copy()
    o.Z = od.whiten(o.A, o.x_ref, o.X)
    total = run_parity(s, o, d, P, n_lag, 3, 3, adopt_shared=True)
    print(f"\n[twisted d=41] parity, {total} accepted", flush=True)
    assert total > 0


def test_local_global_on_a_twisted_target():
    # per-chain factors (M = 2) with the non-Gaussian pi_6 target and inflation
    d, P, n_lag, M = 40, 6, 10, 2
    t = synth.twisted_target(d, 11, 2.0)
    x0 = synth.twisted_exact_draws(t, P, 12)
    s = diam.Sampler(diam.make_config(d, P, n_lag, "fp64", beta=0.4, alpha=1.3, seed=5, M=M), dev(t.mu), dev(t.R),
                     dev(x0.T), twist=dev(t.c))
    o = od.DiamOracle(lambda X: ot.twisted_logpdf(t.R, t.mu, t.c, X), d, P, n_lag, 0.4, alpha=1.3, X=x0, M=M)
    S0, m0 = synth.twisted_warm_moments(t)
    assert s.seed_moments(dev(S0), dev(m0), 2 * P * n_lag)[0] == diam.OK
    assert o.seed_moments(S0, m0, 2 * P * n_lag) == od.OK
    o.A = host(s.get_f64(diam.F_L, (d, d))).T.copy()
    o.Z = od.whiten(o.A, o.x_ref, o.X)
    total = run_parity(s, o, d, P, n_lag, 5, 4, adopt_shared=True)
    print(f"\n[M=2 twisted d={d}] parity, {total} accepted", flush=True)
    assert total > 0
