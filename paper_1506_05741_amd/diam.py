"""Thin ctypes binding of libdiam (include/diam.h).

Argument marshalling only: every step of the sampler runs in the HIP
kernels of ``libdiam.so``.  PyTorch supplies device memory (the workspace and
all caller buffers) and the stream.  ``load()`` raises when the library is
missing; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdiam.so")

FP64, FP32, MIXED = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "mixed": MIXED}

OK, E_ARG, E_STATE, E_HIP, E_NOT_PD, E_TARGET = 0, -1, -2, -3, -4, -5

(F_X, F_Z, F_LOGP, F_ZQ, F_XREF, F_L, F_S, F_M, F_XI, F_LA, F_ACC, F_NACC, F_W, F_WLO, F_U,
 F_SURR, F_NPASS, F_MLP_PARAMS, F_MLP_GRAD, F_MLP_BATCH, F_MLP_STATS, F_LP, F_XREFP) = range(23)

TGT_GAUSS, TGT_LOGREG = 0, 1
PROPOSALS = {"diam": 0, "am": 1, "pcn": 2, "rw": 3}
MLP_HIDDEN = 256

EXPORTED = (
    "diam_workspace_bytes", "diam_init", "diam_step_batch", "diam_merge_moments", "diam_update_proposal",
    "diam_seed_moments", "diam_set_trace", "diam_field_bytes", "diam_get", "diam_get_stats",
    "diam_last_error", "diam_destroy", "diam_profile_enable", "diam_profile_read",
    "diam_surrogate_train", "diam_surrogate_eval", "diam_set_delayed_acceptance",
    "diam_set_beta_adaptation", "diam_psrf_enable", "diam_psrf", "diam_moment_error",
    "diam_moment_error_noalloc",
    "diam_batch_workspace_bytes", "diam_batch_init", "diam_batch_seed_moments", "diam_batch_window",
    "diam_batch_set_tiles", "diam_batch_autotune", "diam_batch_set_graph", "diam_batch_set_persistent",
    "diam_batch_field_bytes",
    "diam_batch_get", "diam_batch_get_stats", "diam_batch_destroy",
)
BATCH_TILES = ("32x2", "64x1", "64x2", "128x2", "32x4")   # target tile rows x k-groups
STAGES = ("rng", "proposal", "target", "step", "merge", "chol", "whiten", "surrogate", "train", "psrf")


class Config(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32), ("P", ctypes.c_int32), ("n_lag", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("beta", ctypes.c_double), ("alpha", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("jitter0", ctypes.c_double), ("jitter_tries", ctypes.c_int32), ("surrogate", ctypes.c_int32),
        ("train_max", ctypes.c_int64), ("proposal", ctypes.c_int32), ("M", ctypes.c_int32),
    ]


class Target(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("mu", ctypes.c_void_p),
                ("R", ctypes.c_void_p), ("A", ctypes.c_void_p), ("y", ctypes.c_void_p), ("n_obs", ctypes.c_int64),
                ("prior_var", ctypes.c_double), ("twist", ctypes.c_void_p)]


class BatchConfig(ctypes.Structure):
    _fields_ = [
        ("G", ctypes.c_int32), ("P", ctypes.c_int32), ("n_lag", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("beta", ctypes.c_double), ("alpha", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("jitter0", ctypes.c_double), ("jitter_tries", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("steps_in_window", ctypes.c_int32), ("last_jitter", ctypes.c_int32),
                ("n_samples", ctypes.c_double), ("windows", ctypes.c_int64), ("last_call_steps", ctypes.c_int64),
                ("beta", ctypes.c_double)]


class DiamError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libdiam status {status}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libdiam.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1506_05741_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    sig = {
        "diam_workspace_bytes": ([ctypes.POINTER(Config), ctypes.POINTER(Target), ctypes.POINTER(sz)], ctypes.c_int),
        "diam_init": ([ctypes.POINTER(vp), ctypes.POINTER(Config), ctypes.POINTER(Target), vp, sz, vp, vp],
                      ctypes.c_int),
        "diam_step_batch": ([vp, i32, vp, vp, vp], ctypes.c_int),
        "diam_merge_moments": ([vp], ctypes.c_int),
        "diam_update_proposal": ([vp, ctypes.POINTER(i32)], ctypes.c_int),
        "diam_seed_moments": ([vp, vp, vp, dbl, ctypes.POINTER(i32)], ctypes.c_int),
        "diam_set_trace": ([vp, vp, i32, vp, i64], ctypes.c_int),
        "diam_field_bytes": ([vp, i32, ctypes.POINTER(sz)], ctypes.c_int),
        "diam_get": ([vp, i32, vp, sz], ctypes.c_int),
        "diam_get_stats": ([vp, ctypes.POINTER(Stats)], ctypes.c_int),
        "diam_last_error": ([], ctypes.c_char_p),
        "diam_destroy": ([vp], None),
        "diam_profile_enable": ([vp, i32], ctypes.c_int),
        "diam_profile_read": ([vp, ctypes.POINTER(dbl), ctypes.POINTER(i64), i32], ctypes.c_int),
        "diam_surrogate_train": ([vp, vp, vp, i64, i32, i32, dbl, ctypes.c_uint64, ctypes.POINTER(dbl)],
                                 ctypes.c_int),
        "diam_surrogate_eval": ([vp, vp, i32, vp], ctypes.c_int),
        "diam_set_delayed_acceptance": ([vp, i32], ctypes.c_int),
        "diam_set_beta_adaptation": ([vp, i32, dbl, dbl, dbl, dbl], ctypes.c_int),
        "diam_psrf_enable": ([vp, i32], ctypes.c_int),
        "diam_psrf": ([vp, vp, ctypes.POINTER(dbl)], ctypes.c_int),
        "diam_moment_error": ([vp, vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl)], ctypes.c_int),
        "diam_moment_error_noalloc": ([vp, vp, i32, vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl), vp],
                                      ctypes.c_int),
        "diam_batch_workspace_bytes": ([ctypes.POINTER(BatchConfig), vp, ctypes.POINTER(sz)], ctypes.c_int),
        "diam_batch_init": ([ctypes.POINTER(vp), ctypes.POINTER(BatchConfig), vp, vp, vp, vp, sz, vp, vp],
                            ctypes.c_int),
        "diam_batch_seed_moments": ([vp, vp, vp, dbl, vp], ctypes.c_int),
        "diam_batch_window": ([vp, vp], ctypes.c_int),
        "diam_batch_set_tiles": ([vp, i32], ctypes.c_int),
        "diam_batch_autotune": ([vp, i32, ctypes.POINTER(i32), vp], ctypes.c_int),
        "diam_batch_set_graph": ([vp, i32], ctypes.c_int),
        "diam_batch_set_persistent": ([vp, i32], ctypes.c_int),
        "diam_batch_field_bytes": ([vp, i32, i32, ctypes.POINTER(sz)], ctypes.c_int),
        "diam_batch_get": ([vp, i32, i32, vp, sz], ctypes.c_int),
        "diam_batch_get_stats": ([vp, ctypes.POINTER(Stats)], ctypes.c_int),
        "diam_batch_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(status):
    if status != OK:
        raise DiamError(status, _lib.diam_last_error().decode())
    return status


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def make_config(d, P, n_lag, precision="fp64", beta=0.3, alpha=1.0, seed=0, jitter0=1e-12, jitter_tries=13,
                surrogate=0, train_max=0, proposal="diam", M=1):
    """surrogate: 0 none, 1 (or True) network surrogate, 2 residual form.
    proposal: "diam", "am", "pcn" or "rw" (the C header's diam_proposal).
    M: intervals of n_lag steps per batch (Section 2.4.1; > 1 gives every
    chain its own factor between global merges)."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    prop = PROPOSALS[proposal] if isinstance(proposal, str) else int(proposal)
    return Config(d, P, n_lag, prec, beta, alpha, seed, jitter0, jitter_tries, int(surrogate), int(train_max),
                  prop, int(M))


def gauss_target(mu, R, twist=None):
    return Target(TGT_GAUSS, 0, _addr(mu), _addr(R), None, None, 0, 0.0, _addr(twist))


def logreg_target(A, y, prior_var):
    n_obs = 0 if A is None else A.shape[0]
    return Target(TGT_LOGREG, 0, None, None, _addr(A), _addr(y), n_obs, float(prior_var), None)


def _addr(t):
    return None if t is None else t.data_ptr()


def workspace_bytes(cfg: Config, tgt: Target) -> int:
    lib = load()
    n = ctypes.c_size_t()
    _check(lib.diam_workspace_bytes(ctypes.byref(cfg), ctypes.byref(tgt), ctypes.byref(n)))
    return n.value


class Sampler:
    """P DIAM chains on the GPU.  Tensors passed in must be CUDA tensors of the
    documented dtype and shape (contiguous); the sampler keeps references.

    Gaussian target: ``Sampler(cfg, mu, R, x0)``.  Logistic regression:
    ``Sampler(cfg, None, None, x0, A=A, y=y, prior_var=v)`` with A (n_obs, d)
    and y (n_obs,) FP32."""

    def __init__(self, cfg: Config, mu, R, x0, stream=None, A=None, y=None, prior_var=None, twist=None):
        """twist (optional, CUDA float64, d): the twisted Gaussians of the paper's test set."""
        import torch
        lib = load()
        self.torch = torch
        self.cfg = cfg
        self.d, self.P = cfg.d, cfg.P
        self.da_on = False
        assert x0.dtype == torch.float64 and x0.is_cuda and x0.numel() == cfg.d * cfg.P and x0.is_contiguous()
        if A is None:
            rdt = torch.float64 if cfg.precision == FP64 else torch.float32
            assert mu.dtype == torch.float64 and mu.is_cuda and mu.numel() == cfg.d and mu.is_contiguous()
            assert R.dtype == rdt and R.is_cuda and R.shape == (cfg.d, cfg.d) and R.is_contiguous()
            if twist is not None:
                assert twist.dtype == torch.float64 and twist.is_cuda and twist.numel() == cfg.d
            self._keep = [mu, R, x0, twist]
            self.tgt = gauss_target(mu, R, twist)
        else:
            assert A.dtype == torch.float32 and A.is_cuda and A.dim() == 2 and A.shape[1] == cfg.d
            assert A.is_contiguous() and y.dtype == torch.float32 and y.is_cuda and y.numel() == A.shape[0]
            self._keep = [A, y, x0]
            self.tgt = logreg_target(A, y, prior_var)
        nbytes = workspace_bytes(cfg, self.tgt)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=x0.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(x0.device)
        ctx = ctypes.c_void_p()
        _check(lib.diam_init(ctypes.byref(ctx), ctypes.byref(cfg), ctypes.byref(self.tgt), _ptr(self.ws),
                             nbytes, _ptr(x0), ctypes.c_void_p(self.stream.cuda_stream)))
        self.ctx = ctx
        self.lib = lib
        self._trace_keep = None

    # -- the sampler's calls ---------------------------------------------------
    def step_batch(self, n_steps, W=None, U=None, n_accepted=None):
        torch = self.torch
        if W is not None:
            assert W.dtype == torch.float64 and W.is_cuda and W.is_contiguous()
            assert W.numel() == self.d * self.P * n_steps
        if U is not None:
            stages = 2 if self.da_on else 1
            assert U.dtype == torch.float64 and U.is_cuda and U.is_contiguous()
            assert U.numel() == self.P * n_steps * stages
        if n_accepted is not None:
            assert n_accepted.dtype == torch.int32 and n_accepted.is_cuda and n_accepted.numel() == self.P
        _check(self.lib.diam_step_batch(self.ctx, int(n_steps), _ptr(W), _ptr(U), _ptr(n_accepted)))

    def merge_moments(self):
        _check(self.lib.diam_merge_moments(self.ctx))

    def update_proposal(self):
        j = ctypes.c_int32()
        st = self.lib.diam_update_proposal(self.ctx, ctypes.byref(j))
        if st not in (OK, E_NOT_PD):
            _check(st)
        return st, j.value

    def seed_moments(self, S0, m0, N0):
        torch = self.torch
        assert S0.dtype == torch.float64 and S0.is_cuda and S0.numel() == self.d * self.d and S0.is_contiguous()
        assert m0.dtype == torch.float64 and m0.is_cuda and m0.numel() == self.d
        self._keep += [S0, m0]
        j = ctypes.c_int32()
        st = self.lib.diam_seed_moments(self.ctx, _ptr(S0), _ptr(m0), float(N0), ctypes.byref(j))
        if st not in (OK, E_NOT_PD):
            _check(st)
        return st, j.value

    def set_trace(self, proj, trace):
        """proj: d x n_proj f64 (column-major, i.e. a (n_proj, d) C-ordered tensor)
        or None; trace: (capacity, 1 + n_proj, P) f64 or None."""
        nproj = 0 if proj is None else proj.numel() // self.d
        cap = 0 if trace is None else trace.shape[0]
        self._trace_keep = (proj, trace)
        _check(self.lib.diam_set_trace(self.ctx, _ptr(proj), nproj, _ptr(trace), cap))

    # -- learned-part form -------------------------------------------------------
    def surrogate_train(self, X, lp, steps, batch=256, lr=1e-3, seed=0):
        """Train the MLP surrogate on pairs X (n, d) f64 CUDA, lp (n,) f64 CUDA;
        returns the mean minibatch loss of the last 50 steps."""
        torch = self.torch
        assert X.dtype == torch.float64 and X.is_cuda and X.is_contiguous() and X.shape[1] == self.d
        assert lp.dtype == torch.float64 and lp.is_cuda and lp.numel() == X.shape[0]
        loss = ctypes.c_double()
        _check(self.lib.diam_surrogate_train(self.ctx, _ptr(X), _ptr(lp), X.shape[0], int(steps), int(batch),
                                             float(lr), int(seed), ctypes.byref(loss)))
        return loss.value

    def surrogate_eval(self, X):
        torch = self.torch
        assert X.dtype == torch.float64 and X.is_cuda and X.is_contiguous() and X.shape[1] == self.d
        out = torch.empty(X.shape[0], dtype=torch.float64, device=X.device)
        _check(self.lib.diam_surrogate_eval(self.ctx, _ptr(X), X.shape[0], _ptr(out)))
        return out

    def set_delayed_acceptance(self, on=True):
        _check(self.lib.diam_set_delayed_acceptance(self.ctx, 1 if on else 0))
        self.da_on = bool(on)

    # -- step-size adaptation (Algorithm 1) ----------------------------------------------
    def set_beta_adaptation(self, on=True, acc_min=0.3, acc_max=0.5, factor=1.2, beta_max=1.0):
        """At every update, beta *= factor (capped) above the acceptance band, /= factor below it."""
        _check(self.lib.diam_set_beta_adaptation(self.ctx, 1 if on else 0, float(acc_min), float(acc_max),
                                                 float(factor), float(beta_max)))

    # -- convergence diagnostic ------------------------------------------------------
    def psrf_enable(self, on=True):
        """Start (zeroing the accumulators) or stop folding merged windows into the PSRF."""
        _check(self.lib.diam_psrf_enable(self.ctx, 1 if on else 0))

    def psrf(self):
        """(sqrt(R_i) for every coordinate as a CUDA float64 tensor, max_i sqrt(R_i) - 1)."""
        torch = self.torch
        out = torch.empty(self.d, dtype=torch.float64, device=self.ws.device)
        worst = ctypes.c_double()
        _check(self.lib.diam_psrf(self.ctx, _ptr(out), ctypes.byref(worst)))
        return out, worst.value

    def moment_error(self, Sigma, mu=None):
        """(|S - m m^T - Sigma|_F / |Sigma|_F, |m - mu|_2 or NaN) of the merged moments."""
        torch = self.torch
        assert Sigma.dtype == torch.float64 and Sigma.is_cuda and Sigma.numel() == self.d * self.d
        assert mu is None or (mu.dtype == torch.float64 and mu.is_cuda and mu.numel() == self.d)
        cov, mean = ctypes.c_double(), ctypes.c_double()
        _check(self.lib.diam_moment_error(self.ctx, _ptr(Sigma.contiguous()), _ptr(mu) if mu is not None else None,
                                          ctypes.byref(cov), ctypes.byref(mean)))
        return cov.value, mean.value

    # -- reading back ------------------------------------------------------------
    def field_bytes(self, field):
        n = ctypes.c_size_t()
        _check(self.lib.diam_field_bytes(self.ctx, field, ctypes.byref(n)))
        return n.value

    def get(self, field):
        """A fresh CUDA uint8 tensor holding the field's bytes (view it with .view(dtype))."""
        torch = self.torch
        n = self.field_bytes(field)
        out = torch.empty(n, dtype=torch.uint8, device=self.ws.device)
        _check(self.lib.diam_get(self.ctx, field, _ptr(out), n))
        return out

    def get_f64(self, field, shape):
        return self.get(field).view(self.torch.float64).reshape(shape)

    def stats(self):
        s = Stats()
        _check(self.lib.diam_get_stats(self.ctx, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def profile(self, on=True):
        _check(self.lib.diam_profile_enable(self.ctx, 1 if on else 0))

    def profile_read(self, reset=False):
        """{stage: (total_ms, regions)} since the last reset."""
        n = len(STAGES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(self.lib.diam_profile_read(self.ctx, ms, cnt, 1 if reset else 0))
        return {STAGES[k]: (ms[k], cnt[k]) for k in range(n)}

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.diam_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def moment_error_noalloc(S, m, Sigma, mu=None, stream=None):
    """Stopping errors of caller-held moments (S (d, d) f64, m (d,) f64 CUDA)
    through diam_moment_error_noalloc: (|S - m m^T - Sigma|_F / |Sigma|_F,
    |m - mu|_2 or NaN).  Runs on the current device's current stream."""
    import torch
    lib = load()
    d = int(m.numel())
    for t in (S, m, Sigma) + ((mu,) if mu is not None else ()):
        assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
    assert S.numel() == d * d and Sigma.numel() == d * d and (mu is None or mu.numel() == d)
    st = stream if stream is not None else torch.cuda.current_stream(m.device)
    cov, mean = ctypes.c_double(), ctypes.c_double()
    _check(lib.diam_moment_error_noalloc(_ptr(S), _ptr(m), d, _ptr(Sigma), _ptr(mu) if mu is not None else None,
                                         ctypes.byref(cov), ctypes.byref(mean), ctypes.c_void_p(st.cuda_stream)))
    return cov.value, mean.value


def _ptr_array(ts, ctype=ctypes.c_void_p):
    return (ctype * len(ts))(*[t.data_ptr() for t in ts])


def batch_workspace_bytes(cfg: BatchConfig, dims) -> int:
    lib = load()
    d = (ctypes.c_int32 * len(dims))(*[int(x) for x in dims])
    n = ctypes.c_size_t()
    _check(lib.diam_batch_workspace_bytes(ctypes.byref(cfg), d, ctypes.byref(n)))
    return n.value


def make_batch_config(G, P, n_lag, beta=0.3, alpha=1.0, seed=0, jitter0=1e-12, jitter_tries=13):
    return BatchConfig(G, P, n_lag, FP32, beta, alpha, seed, jitter0, jitter_tries, 0)


class Batch:
    """G independent Gaussian problems (mu[g] f64 (d_g,), R[g] f32 (d_g, d_g),
    x0[g] f64 (P, d_g) i.e. d_g x P column-major), P chains each."""

    def __init__(self, cfg: BatchConfig, mus, Rs, x0s, stream=None):
        import torch
        lib = load()
        self.torch, self.lib, self.cfg = torch, lib, cfg
        self.G, self.P, self.n = cfg.G, cfg.P, cfg.n_lag
        self.dims = [int(m.numel()) for m in mus]
        assert len(self.dims) == cfg.G == len(Rs) == len(x0s)
        for m, R, x, d in zip(mus, Rs, x0s, self.dims):
            assert m.dtype == torch.float64 and m.is_cuda and m.is_contiguous()
            assert R.dtype == torch.float32 and R.is_cuda and R.is_contiguous() and R.shape == (d, d)
            assert x.dtype == torch.float64 and x.is_cuda and x.is_contiguous() and x.numel() == d * cfg.P
        self._keep = [list(mus), list(Rs), list(x0s)]
        dims = (ctypes.c_int32 * cfg.G)(*self.dims)
        nbytes = batch_workspace_bytes(cfg, self.dims)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=x0s[0].device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(x0s[0].device)
        ctx = ctypes.c_void_p()
        _check(lib.diam_batch_init(ctypes.byref(ctx), ctypes.byref(cfg), dims, _ptr_array(mus), _ptr_array(Rs),
                                   _ptr(self.ws), nbytes, _ptr_array(x0s), ctypes.c_void_p(self.stream.cuda_stream)))
        self.ctx = ctx

    def seed_moments(self, S0s, m0s, N0):
        self._keep.append((list(S0s), list(m0s)))
        j = (ctypes.c_int32 * self.G)()
        st = self.lib.diam_batch_seed_moments(self.ctx, _ptr_array(S0s), _ptr_array(m0s), float(N0), j)
        if st not in (OK, E_NOT_PD):
            _check(st)
        return st, list(j)

    def window(self):
        j = (ctypes.c_int32 * self.G)()
        st = self.lib.diam_batch_window(self.ctx, j)
        if st not in (OK, E_NOT_PD):
            _check(st)
        return st, list(j)

    def set_tiles(self, choice):
        _check(self.lib.diam_batch_set_tiles(self.ctx, int(choice)))

    def set_graph(self, on=True):
        _check(self.lib.diam_batch_set_graph(self.ctx, 1 if on else 0))

    def set_persistent(self, on=True):
        _check(self.lib.diam_batch_set_persistent(self.ctx, 1 if on else 0))

    def autotune(self, reps=20):
        c = ctypes.c_int32()
        us = (ctypes.c_double * len(BATCH_TILES))()
        _check(self.lib.diam_batch_autotune(self.ctx, int(reps), ctypes.byref(c), us))
        return c.value, dict(zip(BATCH_TILES, list(us)))

    def get(self, g, field):
        torch = self.torch
        n = ctypes.c_size_t()
        _check(self.lib.diam_batch_field_bytes(self.ctx, int(g), field, ctypes.byref(n)))
        out = torch.empty(n.value, dtype=torch.uint8, device=self.ws.device)
        _check(self.lib.diam_batch_get(self.ctx, int(g), field, _ptr(out), n.value))
        return out

    def get_f64(self, g, field, shape):
        return self.get(g, field).view(self.torch.float64).reshape(shape)

    def stats(self):
        s = Stats()
        _check(self.lib.diam_batch_get_stats(self.ctx, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.diam_batch_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
