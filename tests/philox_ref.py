"""Philox4x32-10 written from its published definition (Salmon et al., SC'11),
used by the tests to check the GPU's draws.  Pinned by the known-answer
vectors in tests/golden/philox4x32_10_kat.txt."""
import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised over numpy uint64 arrays holding 32-bit values."""
    c = [np.asarray(x, dtype=np.uint64) & MASK for x in (c0, c1, c2, c3)]
    k0 = np.uint64(k0) & np.uint64(MASK)
    k1 = np.uint64(k1) & np.uint64(MASK)
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(W0)) & np.uint64(MASK)
            k1 = (k1 + np.uint64(W1)) & np.uint64(MASK)
        p0 = np.uint64(M0) * c[0]
        p1 = np.uint64(M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def u01_f64(a, b):
    k = ((np.asarray(a, dtype=np.uint64) << np.uint64(32)) | np.asarray(b, dtype=np.uint64)) >> np.uint64(12)
    return (k.astype(np.float64) + 0.5) * 2.0 ** -52


def gpu_uniforms(seed, s0, n, P):
    """The library's uniforms for steps [s0, s0+n): U[t][p]."""
    t = np.arange(n, dtype=np.uint64)[:, None] + np.uint64(s0)
    p = np.arange(P, dtype=np.uint64)[None, :]
    st = np.broadcast_to(t, (n, P))
    r = philox4x32_10(st & np.uint64(MASK), st >> np.uint64(32), np.full((n, P), 1, np.uint64), p >> np.uint64(1),
                      seed & MASK, seed >> 32)
    odd = (p & np.uint64(1)).astype(bool)
    return np.where(odd, u01_f64(r[2], r[3]), u01_f64(r[0], r[1]))


def gpu_normals_f64(seed, s0, n, d, P):
    """The library's FP64 normals for steps [s0, s0+n): W[t] as (n, P, d)."""
    total = n * P * d
    q = np.arange((total + 1) // 2, dtype=np.uint64)
    ctr = np.uint64(s0 * P * d) + np.uint64(2) * q
    r = philox4x32_10(ctr & np.uint64(MASK), ctr >> np.uint64(32), 0, 0, seed & MASK, seed >> 32)
    u1, u2 = u01_f64(r[0], r[1]), u01_f64(r[2], r[3])
    rad = np.sqrt(-2.0 * np.log(u1))
    out = np.empty(2 * q.size)
    out[0::2] = rad * np.cos(2 * np.pi * u2)
    out[1::2] = rad * np.sin(2 * np.pi * u2)
    return out[:total].reshape(n, P, d)
