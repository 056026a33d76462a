"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).

The eigensolver draws random vectors in two places: the start vector of an
extension (Alg. 4 first step) and the replacement vector after a Lanczos
breakdown (Alg. 3).  Both sides of the parity check draw them from this
published generator, so the random numbers are identical bit for bit.

Vector entry i of draw number ``call`` at level ``level`` with 64-bit ``seed``:
counter = (i // 2, call, level, 0), key = (seed & 0xffffffff, seed >> 32);
the four output words (x0, x1, x2, x3) give entry 2c from (x0, x1) and entry
2c+1 from (x2, x3) as  ((xa >> 5) * 2^26 + (xb >> 6)) * 2^-53 - 0.5,
an exactly representable double in [-0.5, 0.5).
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint32(0x9E3779B9)
_W1 = np.uint32(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Vectorised Philox4x32 with 10 rounds.

    ctr: uint32 array [..., 4]; key: uint32 array [..., 2].  Returns uint32 [..., 4].
    """
    c = np.array(ctr, dtype=np.uint32, copy=True)
    k = np.array(key, dtype=np.uint32, copy=True)
    c0, c1, c2, c3 = (c[..., i].astype(np.uint64) for i in range(4))
    k0 = k[..., 0].astype(np.uint64)
    k1 = k[..., 1].astype(np.uint64)
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(_W0)) & _MASK
            k1 = (k1 + np.uint64(_W1)) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & _MASK, lo1, (hi0 ^ c3 ^ k1) & _MASK, lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def uniform_vector(n: int, seed: int, level: int, call: int) -> np.ndarray:
    """Length-n float64 vector with entries in [-0.5, 0.5) (see module doc)."""
    nc = (n + 1) // 2
    ctr = np.zeros((nc, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(nc, dtype=np.uint64).astype(np.uint32)
    ctr[:, 1] = np.uint32(call & 0xFFFFFFFF)
    ctr[:, 2] = np.uint32(level & 0xFFFFFFFF)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)
    out = philox4x32_10(ctr, np.broadcast_to(key, (nc, 2)))
    x = out.astype(np.uint64)
    a = ((x[:, 0] >> np.uint64(5)).astype(np.float64) * 67108864.0
         + (x[:, 1] >> np.uint64(6)).astype(np.float64)) / 9007199254740992.0
    b = ((x[:, 2] >> np.uint64(5)).astype(np.float64) * 67108864.0
         + (x[:, 3] >> np.uint64(6)).astype(np.float64)) / 9007199254740992.0
    v = np.empty(2 * nc)
    v[0::2] = a
    v[1::2] = b
    return v[:n] - 0.5
