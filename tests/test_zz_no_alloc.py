"""The entry point for callers that cannot allocate (diam_moment_error_noalloc)
against diam_moment_error, through the C ABI: the same kernels on the same
moments, so the stopping errors must be bitwise equal.  Two calls in a row on
one GPU (the static partials keep the first call's contents), the second with
a smaller input; then argument checks."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1506_05741_amd import diam, synth


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def sampler_after_windows(d, P, n_lag, windows, seed):
    t = synth.gaussian_target(d, seed)
    x0 = synth.gaussian_exact_draws(t, P, seed + 1)
    s = diam.Sampler(diam.make_config(d, P, n_lag, "fp64", seed=seed), dev(t.mu), dev(t.R), dev(x0.T))
    S0, m0 = synth.gaussian_warm_moments(t)
    assert s.seed_moments(dev(S0), dev(m0), 3 * P * n_lag)[0] == diam.OK
    for _ in range(windows):
        s.step_batch(n_lag)
        s.merge_moments()
        assert s.update_proposal()[0] == diam.OK
    return t, s


@pytest.mark.parametrize("sizes", [(300, 40)])
def test_noalloc_moment_error_equals_the_context_call(sizes):
    for d in sizes:                     # the second call is smaller than the first
        t, s = sampler_after_windows(d, 8, 10, 3, 40 + d)
        Sig, mu = dev(t.Sigma), dev(t.mu)
        ref = s.moment_error(Sig, mu)
        S = s.get_f64(diam.F_S, (d, d)).contiguous()
        m = s.get_f64(diam.F_M, (d,)).contiguous()
        got = diam.moment_error_noalloc(S, m, Sig, mu)
        print(f"\nd={d}: context call {ref}, no-alloc call {got}", flush=True)
        assert got == ref and np.isfinite(got[0]) and got[0] > 0
        got_nomu = diam.moment_error_noalloc(S, m, Sig)
        assert got_nomu[0] == ref[0] and np.isnan(got_nomu[1])
        # the errors themselves: the definition on the host (FP64, any order)
        Sh, mh = S.cpu().numpy().T, m.cpu().numpy()
        C = Sh - np.outer(mh, mh)
        cov = np.linalg.norm(C - t.Sigma) / np.linalg.norm(t.Sigma)
        assert abs(got[0] - cov) <= 1e-12 * cov + 1e-15
        assert abs(got[1] - np.linalg.norm(mh - t.mu)) <= 1e-12 * np.linalg.norm(mh - t.mu) + 1e-15
        s.close()


def test_noalloc_moment_error_rejects_bad_arguments():
    d = 4
    z = torch.zeros(d * d, dtype=torch.float64, device="cuda")
    lib = diam.load()
    import ctypes
    cov, mean = ctypes.c_double(), ctypes.c_double()
    st = lib.diam_moment_error_noalloc(ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(z.data_ptr()), 0,
                                       ctypes.c_void_p(z.data_ptr()), None, ctypes.byref(cov), ctypes.byref(mean),
                                       None)
    assert st == diam.E_ARG and b"d = 0" in lib.diam_last_error()
    st = lib.diam_moment_error_noalloc(None, ctypes.c_void_p(z.data_ptr()), d, ctypes.c_void_p(z.data_ptr()), None,
                                       ctypes.byref(cov), ctypes.byref(mean), None)
    assert st == diam.E_ARG
