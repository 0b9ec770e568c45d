"""The C-ABI library loads on the host and exports every symbol the header
declares; host-only calls validate their arguments.  No GPU needed."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1506_05741_amd import diam

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "diam.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(diam_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(diam.LIB_PATH)
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(diam.EXPORTED) == names


def test_binding_loads():
    lib = diam.load()
    assert lib.diam_last_error() is not None


# host-only size queries check that the target's pointers are set, never
# dereference them: placeholders stand in for device buffers
GAUSS = diam.Target(diam.TGT_GAUSS, 0, 256, 512, None, None, 0, 0.0)


def logreg(n_obs=1000, prior_var=10.0):
    return diam.Target(diam.TGT_LOGREG, 0, None, None, 256, 512, n_obs, prior_var)


def test_workspace_bytes_scales_with_precision():
    big = diam.workspace_bytes(diam.make_config(4096, 256, 256, "fp64"), GAUSS)
    mix = diam.workspace_bytes(diam.make_config(4096, 256, 256, "mixed"), GAUSS)
    assert 6 * 2 ** 30 < big < 8 * 2 ** 30
    assert mix < 0.6 * big
    assert diam.workspace_bytes(diam.make_config(1, 1, 1), GAUSS) > 0


def test_workspace_bytes_of_the_local_global_form():
    # M > 1 adds ten regions (each a 256-byte placeholder otherwise): per-chain
    # factors, local sums G_p and h_p, pivots, one chain's S_pg and m_pg, all
    # chains' covariances and pivots, status words, block inverses (64 x 64
    # per block of 64 rows)
    d, P = 64, 4
    base = diam.workspace_bytes(diam.make_config(d, P, 4, "fp64"), GAUSS)
    lg = diam.workspace_bytes(diam.make_config(d, P, 4, "fp64", M=3), GAUSS)
    sizes = [P * d * d * 8, P * d * d * 8, d * P * 8, d * P * 8, d * d * 8, d * 8, P * d * d * 8, d * P * 8, P * 4,
             P * 64 * 64 * 8]
    assert lg - base == sum((b + 255) // 256 * 256 for b in sizes) - 10 * 256


def test_workspace_bytes_of_the_learned_form():
    cfg = diam.make_config(512, 256, 64, "fp32")
    base = diam.workspace_bytes(cfg, logreg(200000))
    # the logistic target's partial sums take one FP64 row per 64 observations
    assert diam.workspace_bytes(cfg, logreg(200064)) - base in range(256 * 8, 256 * 8 + 512)
    sur = diam.workspace_bytes(diam.make_config(512, 256, 64, "fp32", surrogate=True, train_max=10000), logreg(200000))
    big = diam.workspace_bytes(diam.make_config(512, 256, 64, "fp32", surrogate=True, train_max=20000), logreg(200000))
    # training pairs are held standardised in FP32: d + 1 floats each
    assert abs((big - sur) - 10000 * 513 * 4) < 4096
    nparam = 256 * 512 + 256 + 256 * 256 + 256 + 256 + 1
    assert sur - base > 5 * nparam * 4 + 10000 * 513 * 4


@pytest.mark.parametrize("tgt,msg", [
    (logreg(n_obs=0), "n_obs"),
    (logreg(prior_var=0.0), "prior_var"),
    (diam.Target(diam.TGT_LOGREG, 0, None, None, None, 512, 10, 1.0), "needs A"),
    (diam.Target(diam.TGT_GAUSS, 0, None, 512, None, None, 0, 0.0), "needs mu"),
    (diam.Target(9, 0, 256, 512, None, None, 0, 0.0), "unknown target"),
])
def test_bad_target_is_rejected(tgt, msg):
    with pytest.raises(diam.DiamError) as e:
        diam.workspace_bytes(diam.make_config(8, 2, 4), tgt)
    assert e.value.status == diam.E_ARG and msg in str(e.value)


@pytest.mark.parametrize("kw,msg", [
    (dict(d=0), "d, P and n_lag"),
    (dict(beta=1.5), "beta"),
    (dict(beta=0.0), "beta"),
    (dict(alpha=0.5), "alpha"),
    (dict(precision=7), "precision"),
    (dict(jitter0=-1.0), "jitter0"),
    (dict(train_max=-5), "train_max"),
    (dict(proposal=9), "unknown proposal"),
    (dict(proposal="rw", surrogate=2, train_max=10), "residual surrogate"),
    (dict(M=-1), "M must be"),
    (dict(M=3, precision="fp32"), "M > 1 needs"),
    (dict(M=3, proposal="am"), "M > 1 needs"),
    (dict(M=3, surrogate=1, train_max=10), "M > 1 needs"),
])
def test_bad_config_is_rejected(kw, msg):
    base = dict(d=8, P=2, n_lag=4, precision="fp64", beta=0.3, alpha=1.0)
    base.update(kw)
    cfg = diam.make_config(**base)
    with pytest.raises(diam.DiamError) as e:
        diam.workspace_bytes(cfg, GAUSS)
    assert e.value.status == diam.E_ARG and msg in str(e.value)


def test_null_arguments_are_rejected():
    lib = diam.load()
    ctx = ctypes.c_void_p()
    cfg = diam.make_config(8, 2, 4)
    st = lib.diam_init(ctypes.byref(ctx), ctypes.byref(cfg), None, None, 0, None, None)
    assert st == diam.E_ARG
    assert lib.diam_step_batch(None, 1, None, None, None) == diam.E_ARG
    assert lib.diam_merge_moments(None) == diam.E_ARG
    assert lib.diam_update_proposal(None, None) == diam.E_ARG
    assert lib.diam_surrogate_train(None, None, None, 0, 0, 0, 0.0, 0, None) == diam.E_ARG
    assert lib.diam_surrogate_eval(None, None, 0, None) == diam.E_ARG
    assert lib.diam_set_delayed_acceptance(None, 1) == diam.E_ARG
    assert b"null" in lib.diam_last_error()


def test_missing_library_fails_loudly(tmp_path):
    saved = diam._lib
    diam._lib = None
    try:
        with pytest.raises(RuntimeError, match="missing"):
            diam.load(str(tmp_path / "libdiam.so"))
    finally:
        diam._lib = saved


def test_philox_reference_matches_published_kat():
    from tests.philox_ref import philox4x32_10
    path = os.path.join(ROOT, "tests", "golden", "philox4x32_10_kat.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox4x32_10(*v[:6])
        assert [int(o) for o in out] == v[6:]


@pytest.mark.parametrize("kw,msg", [
    (dict(n_lag=7), "n_lag must be even"),
    (dict(P=64, n_lag=128), "P * n_lag"),
    (dict(G=0), "G must"),
    (dict(beta=0.0), "beta"),
])
def test_bad_batch_config_is_rejected(kw, msg):
    base = dict(G=3, P=32, n_lag=8)
    base.update(kw)
    G = base.pop("G")
    cfg = diam.make_batch_config(G, **base)
    with pytest.raises(diam.DiamError) as e:
        diam.batch_workspace_bytes(cfg, [16] * max(G, 1))
    assert e.value.status == diam.E_ARG and msg in str(e.value)


def test_batch_rejects_other_precisions_and_bad_dims():
    cfg = diam.make_batch_config(2, 32, 8)
    cfg.precision = diam.FP64
    with pytest.raises(diam.DiamError, match="DIAM_FP32 only"):
        diam.batch_workspace_bytes(cfg, [16, 16])
    with pytest.raises(diam.DiamError, match="outside"):
        diam.batch_workspace_bytes(diam.make_batch_config(2, 32, 8), [16, 0])


def test_batch_workspace_grows_with_the_problems():
    cfg = diam.make_batch_config(2, 32, 8)
    a = diam.batch_workspace_bytes(cfg, [64, 64])
    b = diam.batch_workspace_bytes(cfg, [64, 128])
    # per problem: five d x d FP64 matrices (S, L, C, scatter) and FP32 factor dominate
    assert b - a > (128 * 128 - 64 * 64) * (4 * 8 + 4)
