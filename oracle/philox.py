"""Counter-based normal deviates for the Langevin step of the path integrator (oracle side).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the benchmark's CPU
baseline, never by the library.

Philox4x64-10 as published by Salmon, Moraes, Dror and Shaw ("Parallel random numbers:
as easy as 1, 2, 3", SC 2011): a 4 x 64-bit counter and a 2 x 64-bit key; each of ten
rounds multiplies counter words 0 and 2 by two fixed odd constants, taking the 128-bit
products apart into high and low words, and recombines them with the other two words
and the round key; the key is advanced by two Weyl increments between rounds.

Normal deviates: each 64-bit output x becomes u = (floor(x / 2^12) + 1/2) 2^-52, exact
in FP64 and inside (0, 1), and pairs (u0, u1) go through the Box-Muller transform
    z0 = sqrt(-2 ln u0) cos(2 pi u1),  z1 = sqrt(-2 ln u0) sin(2 pi u1).
One Philox call per (bead, atom) gives the three Cartesian deviates: z0, z1 from
outputs 0 and 1, z2 from outputs 2 and 3.  The counter is (bead * Q + atom, step, 0, 0)
and the key (seed, 0).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def mulhilo64(a, b):
    """High and low 64-bit words of the 128-bit product of uint64 arrays a and b."""
    a = np.asarray(a, np.uint64)
    b = np.asarray(b, np.uint64)
    al, ah = a & _M32, a >> _S32
    bl, bh = b & _M32, b >> _S32
    p0, p1, p2, p3 = al * bl, al * bh, ah * bl, ah * bh
    mid = (p0 >> _S32) + (p1 & _M32) + (p2 & _M32)
    hi = p3 + (p1 >> _S32) + (p2 >> _S32) + (mid >> _S32)
    with np.errstate(over="ignore"):
        lo = a * b
    return hi, lo


def philox4x64_10(ctr, key):
    """ctr: (..., 4) uint64, key: (..., 2) uint64 -> (..., 4) uint64."""
    c = [np.array(ctr[..., k], np.uint64) for k in range(4)]
    k0 = np.array(key[..., 0], np.uint64)
    k1 = np.array(key[..., 1], np.uint64)
    with np.errstate(over="ignore"):
        for r in range(10):
            hi0, lo0 = mulhilo64(M0, c[0])
            hi1, lo1 = mulhilo64(M1, c[2])
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
            if r < 9:
                k0 = k0 + W0
                k1 = k1 + W1
    return np.stack(c, axis=-1)


def uniform52(x):
    """(floor(x / 2^12) + 1/2) * 2^-52: exactly representable, inside (0, 1)."""
    return ((np.asarray(x, np.uint64) >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0 ** -52


def box_muller(u0, u1):
    rho = np.sqrt(-2.0 * np.log(u0))
    return rho * np.cos(2.0 * np.pi * u1), rho * np.sin(2.0 * np.pi * u1)


def path_normals(seed, step, N, Q):
    """Standard normal deviates [N][Q][3] for the Langevin step `step` of a path."""
    idx = np.arange(N * Q, dtype=np.uint64)
    ctr = np.zeros((N * Q, 4), np.uint64)
    ctr[:, 0] = idx
    ctr[:, 1] = np.uint64(step)
    key = np.zeros((N * Q, 2), np.uint64)
    key[:, 0] = np.uint64(seed)
    x = philox4x64_10(ctr, key)
    u = uniform52(x)
    z0, z1 = box_muller(u[:, 0], u[:, 1])
    z2, _ = box_muller(u[:, 2], u[:, 3])
    return np.stack([z0, z1, z2], axis=-1).reshape(N, Q, 3)
