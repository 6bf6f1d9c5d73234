"""Ewald summation of periodic Coulomb interactions -- FP64, TEST INFRASTRUCTURE ONLY.

The paper's standard MD runs (Appendix A.1) treat long-range electrostatics with
particle-mesh Ewald (PME) and a 1.2 nm real-space cut-off.  PME approximates the Ewald sum;
this module is the Ewald sum itself, written out from its textbook definition, and the
yardstick the oracle's PME (pme.py) is pinned against.

For charges q_i at x_i in an orthorhombic box of volume V, splitting parameter beta
and Coulomb factor f (kJ mol^-1 nm e^-2, divided by eps_r):

  E_real  = f sum_{i<j, not excluded, r_ij < r_c} q_i q_j erfc(beta r_ij) / r_ij
            (minimum image; beta is chosen so that erfc(beta r_c) is negligible)
  E_recip = f / (2 pi V) sum_{m != 0} exp(-pi^2 |m|^2 / beta^2) / |m|^2 |S(m)|^2,
            m = (m_x/L_x, m_y/L_y, m_z/L_z) with integer m_a,
            S(m) = sum_j q_j exp(2 pi i m . x_j)
  E_self  = -f beta / sqrt(pi) sum_i q_i^2
  E_excl  = -f sum_{excluded i<j} q_i q_j erf(beta r_ij) / r_ij
            (the reciprocal sum contains every pair; this removes excluded pairs)
  E_bg    = -f pi (sum_i q_i)^2 / (2 V beta^2)      (neutralising background)

The total does not depend on beta (up to the real-space truncation), which is one of
the pins of this module; the others are the Madelung constants of rock salt and of
caesium chloride, and the identity that excluding a pair removes exactly its bare
Coulomb term f q_i q_j / r_ij.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf, erfc

from .potential import min_image


def beta_from_rtol(rc, rtol):
    """The splitting parameter with erfc(beta r_c) = rtol (bisection in FP64)."""
    lo, hi = 0.0, 1.0
    while math.erfc(hi * rc) > rtol:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if math.erfc(mid * rc) > rtol:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def recip_mmax(beta, box, tol=1e-18):
    """Per-axis integer bound on m so that every omitted term has
    exp(-pi^2 |m|^2 / beta^2) below tol."""
    mlen = beta * math.sqrt(-math.log(tol)) / math.pi   # |m| in nm^-1
    return [int(math.ceil(mlen * L)) for L in box]


def _mvectors(box, mmax):
    ax = [np.arange(-n, n + 1) for n in mmax]
    M = np.stack(np.meshgrid(*ax, indexing="ij"), -1).reshape(-1, 3)
    M = M[np.any(M != 0, axis=1)]
    return M / np.asarray(box, np.float64)


def structure_factor(X, q, mvec):
    """S(m) = sum_j q_j exp(2 pi i m . x_j) for every row of mvec."""
    return np.exp(2j * np.pi * (mvec @ np.asarray(X, np.float64).T)) @ q


def recip_energy(X, q, box, beta, f, mmax=None, chunk=4096):
    """E_recip as the plain lattice sum over m != 0."""
    box = np.asarray(box, np.float64)
    V = float(np.prod(box))
    mvec = _mvectors(box, mmax or recip_mmax(beta, box))
    e = 0.0
    for a in range(0, len(mvec), chunk):
        m = mvec[a:a + chunk]
        m2 = np.einsum("ak,ak->a", m, m)
        S = structure_factor(X, q, m)
        e += float(np.sum(np.exp(-np.pi ** 2 * m2 / beta ** 2) / m2 * np.abs(S) ** 2))
    return f * e / (2.0 * np.pi * V)


def recip_forces(X, q, box, beta, f, mmax=None, chunk=4096):
    """-grad E_recip: F_i = (2 f q_i / V) sum_m exp(-pi^2 m^2/beta^2)/m^2 m
    Im[exp(2 pi i m . x_i) conj(S(m))]  (differentiating |S(m)|^2 = S conj(S))."""
    X = np.asarray(X, np.float64)
    box = np.asarray(box, np.float64)
    V = float(np.prod(box))
    mvec = _mvectors(box, mmax or recip_mmax(beta, box))
    F = np.zeros_like(X)
    for a in range(0, len(mvec), chunk):
        m = mvec[a:a + chunk]
        m2 = np.einsum("ak,ak->a", m, m)
        ph = np.exp(2j * np.pi * (X @ m.T))              # (Q, M)
        S = ph.T @ q                                     # (M,)
        w = np.exp(-np.pi ** 2 * m2 / beta ** 2) / m2
        F += (np.imag(ph * np.conj(S)[None, :]) * w[None, :]) @ m
    return 2.0 * f * q[:, None] * F / V


def real_energy(X, q, box, beta, rc, f, excluded=()):
    """E_real over minimum-image pairs i < j within r_c that are not excluded."""
    X = np.asarray(X, np.float64)
    ex = {(min(i, j), max(i, j)) for i, j in excluded}
    e = 0.0
    Q = len(q)
    for i in range(Q - 1):
        d = min_image(X[i + 1:] - X[i], box)
        r = np.sqrt(np.einsum("ak,ak->a", d, d))
        for k in np.nonzero(r < rc)[0]:
            j = i + 1 + int(k)
            if (i, j) not in ex:
                e += q[i] * q[j] * math.erfc(beta * r[k]) / r[k]
    return f * e


def self_energy(q, beta, f):
    return -f * beta / math.sqrt(math.pi) * float(np.sum(np.asarray(q) ** 2))


def background_energy(q, box, beta, f):
    V = float(np.prod(box))
    return -f * math.pi * float(np.sum(q)) ** 2 / (2.0 * V * beta ** 2)


def exclusion_energy(X, q, box, beta, f, excluded=()):
    """E_excl = -f sum_{excluded} q_i q_j erf(beta r) / r (minimum image)."""
    e = 0.0
    for i, j in excluded:
        d = min_image(np.asarray(X[j]) - np.asarray(X[i]), box)
        r = float(np.sqrt(d @ d))
        e -= q[i] * q[j] * float(erf(beta * r)) / r
    return f * e


def ewald_energy(X, q, box, beta, rc, f, excluded=(), mmax=None):
    """Total Ewald electrostatic energy and its parts (dict)."""
    q = np.asarray(q, np.float64)
    box = np.asarray(box, np.float64)
    parts = dict(
        real=real_energy(X, q, box, beta, rc, f, excluded),
        recip=recip_energy(X, q, box, beta, f, mmax),
        self=self_energy(q, beta, f),
        excl=exclusion_energy(X, q, box, beta, f, excluded),
        bg=background_energy(q, box, beta, f),
    )
    parts["total"] = sum(parts.values())
    return parts


# pair functions of the real-space term for r as numpy arrays (psi = erfc(beta r)/r)

def psi(r, beta):
    return erfc(beta * r) / r


def psi_d1(r, beta):
    D = 2.0 * beta / math.sqrt(math.pi) * np.exp(-(beta * r) ** 2)
    return -erfc(beta * r) / r ** 2 - D / r


def psi_d2(r, beta):
    D = 2.0 * beta / math.sqrt(math.pi) * np.exp(-(beta * r) ** 2)
    return 2.0 * erfc(beta * r) / r ** 3 + D * (2.0 / r ** 2 + 2.0 * beta ** 2)


def chi(r, beta):
    """erf(beta r)/r, the excluded-pair correction (finite at r = 0)."""
    return erf(beta * r) / r


def chi_d1(r, beta):
    D = 2.0 * beta / math.sqrt(math.pi) * np.exp(-(beta * r) ** 2)
    return D / r - erf(beta * r) / r ** 2


def chi_d2(r, beta):
    D = 2.0 * beta / math.sqrt(math.pi) * np.exp(-(beta * r) ** 2)
    return -2.0 * beta ** 2 * D - 2.0 * D / r ** 2 + 2.0 * erf(beta * r) / r ** 3
