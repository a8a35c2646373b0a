"""Control-noise generator for the oracle (test infrastructure only).

Alg. 1, Step 1 draws eps_k^s ~ N(0, Sigma_sim) for every sample s and step k,
and Eq. (8) keeps controls in [u_min, u_max].  The draw is made reproducible
and identical on every side by a counter-based generator:

* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11): a 4x32-bit counter and a 2x32-bit key; each of the
  ten rounds multiplies counter words 0 and 2 by two fixed odd constants and
  mixes the high halves with the other words and the key; the key advances by
  two Weyl constants between rounds.
* counter = (k, s, pid, tag), key = (seed mod 2^32, seed >> 32).
* uniforms u = ((word >> 9) + 1/2) * 2^-23 from output words 0 and 1: every
  value is a multiple of 2^-24 below 1, so it is exact in binary32 and binary64
  alike, and it is never 0 or 1.
* Box-Muller: z0 = sqrt(-2 ln u1) cos(2 pi u2), z1 = sqrt(-2 ln u1) sin(2 pi u2).
"""
from __future__ import annotations

import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
_MUL = (np.uint64(0xD2511F53), np.uint64(0xCD9E8D57))
_WEYL = (np.uint64(0x9E3779B9), np.uint64(0xBB67AE85))


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds.

    ctr: integer array [..., 4] of 32-bit counter words; key: (k0, k1).
    Returns uint32 array [..., 4].
    """
    ctr = np.asarray(ctr, dtype=np.uint64)
    x0, x1, x2, x3 = (ctr[..., i] & _MASK for i in range(4))
    k0 = np.uint64(int(key[0]) & 0xFFFFFFFF)
    k1 = np.uint64(int(key[1]) & 0xFFFFFFFF)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _WEYL[0]) & _MASK
            k1 = (k1 + _WEYL[1]) & _MASK
        p0 = _MUL[0] * x0          # < 2^64: exact in uint64
        p1 = _MUL[1] * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        x0, x1, x2, x3 = (hi1 ^ x1 ^ k0), lo1, (hi0 ^ x3 ^ k1), lo0
    return np.stack([x0, x1, x2, x3], axis=-1).astype(np.uint32)


def seed_key(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & 0xFFFFFFFF, seed >> 32)


def uniform_open(word) -> np.ndarray:
    """((w >> 9) + 0.5) * 2^-23 in float64 (exact)."""
    w = np.asarray(word, dtype=np.uint64) >> np.uint64(9)
    return (w.astype(np.float64) + 0.5) * 2.0 ** -23


def box_muller(u1, u2):
    r = np.sqrt(-2.0 * np.log(u1))
    a = 2.0 * np.pi * u2
    return r * np.cos(a), r * np.sin(a)


def standard_normals(k: int, sample_ids, seed: int, pid: int = 0, tag: int = 0):
    """The pair of N(0,1) draws for step k of the given sample ids."""
    s = np.asarray(sample_ids, dtype=np.uint64)
    n = s.shape[0]
    ctr = np.stack([np.full(n, k, np.uint64), s, np.full(n, pid, np.uint64),
                    np.full(n, tag, np.uint64)], axis=-1)
    w = philox4x32_10(ctr, seed_key(seed))
    return box_muller(uniform_open(w[:, 0]), uniform_open(w[:, 1]))


def sampled_controls(U, sample_ids, seed: int, sig, u_min, u_max, pid: int = 0) -> np.ndarray:
    """u^s(k) = clip(u(k) + eps_k^s) for all k < T and the given samples -> [T, n, 2].

    Alg. 1, Step 1: eps_k^s ~ N(0, diag(sig_v^2, sig_w^2)); Eq. (8): box.
    """
    U = np.asarray(U, dtype=np.float64)
    T = U.shape[0]
    out = np.empty((T, len(sample_ids), 2))
    for k in range(T):
        z0, z1 = standard_normals(k, sample_ids, seed, pid)
        out[k, :, 0] = np.clip(U[k, 0] + sig[0] * z0, u_min[0], u_max[0])
        out[k, :, 1] = np.clip(U[k, 1] + sig[1] * z1, u_min[1], u_max[1])
    return out
