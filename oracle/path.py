"""Effective path potential, its gradient, and the paper's effective forces -- FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring): no product code imports this.

Notation follows section 1.1 of the paper.  A discretised trajectory of N steps is a
polymer of beads R^1 .. R^N (eq. 3).  Per atom i:

    K_i = m_i nu / (2 dt)          spring constant (section 1.1, below eq. 3)
    c_i = dt / (m_i nu)            so that the rest length is L^n = c F^n

Reading of the rest length: the text prints L^n = (m nu / dt) F^n, which is not a
length; the effective forces of eqs. (5)-(7) are the gradient of eq. (3) only when
L^n = (dt / (m nu)) F^n, i.e. K_i c_i = 1/2.  That is the reading used here.

    d^n = mi(R^{n+1} - R^n) - c F(R^n),   n = 1 .. N-1     (eta^n of eq. 5 / kernel 1
                                                            of section 2.1; mi = minimum image)
    V_eff = U(R^1) + sum_n sum_i K_i/2 |d^n_i|^2            (eq. 3; kernel 7 is the sum)

Exact gradient G^n = grad_{R^n} V_eff (from d d^n/d R^n = -I + C H, d d^n/d R^{n+1} = I):

    G^n = -[n = 1] F^1 + [n >= 2] K d^{n-1} + [n <= N-1] (-K d^n + 1/2 H(R^n) d^n)

and F_eff^n = -G^n reproduces eqs. (5)-(7) once the finite-difference term of eq. (5)
is replaced by its limit -1/2 H d^n.
"""
from __future__ import annotations

import numpy as np

from .potential import min_image


def coefficients(model):
    """(c, K) per atom, each of shape (Q,)."""
    c = model.dt / (model.mass * model.nu)
    K = model.mass * model.nu / (2.0 * model.dt)
    return c, K


def residuals(model, R, forces=None):
    """d^n for n = 1..N-1 as an (N-1, Q, 3) array, and the forces F^n used for them.
    `forces` may supply precomputed F(R^n) for n = 1..N-1."""
    R = np.asarray(R, np.float64)
    N = R.shape[0]
    c, _ = coefficients(model)
    if forces is not None:
        F = forces
    elif N > 1:
        F = np.stack([model.forces(R[n]) for n in range(N - 1)])
    else:
        F = np.zeros((0, model.Q, 3))
    d = np.empty((max(N - 1, 0), model.Q, 3))
    for n in range(N - 1):
        d[n] = min_image(R[n + 1] - R[n], model.box) - c[:, None] * F[n]
    return d, F


def veff(model, R):
    """(V_eff, U(R^1), spring energy) of eq. (3)."""
    R = np.asarray(R, np.float64)
    _, K = coefficients(model)
    u1 = model.energy(R[0])
    d, _ = residuals(model, R)
    es = float(np.sum(0.5 * K[None, :, None] * d * d)) if d.size else 0.0
    return u1 + es, u1, es


def veff_grad(model, R):
    """Exact gradient G (N, Q, 3) of V_eff and the value V_eff."""
    R = np.asarray(R, np.float64)
    N = R.shape[0]
    _, K = coefficients(model)
    F1 = model.forces(R[0])
    Fs = np.stack([F1] + [model.forces(R[n]) for n in range(1, N - 1)]) if N > 1 else None
    d, _ = residuals(model, R, Fs)
    G = np.zeros_like(R)
    G[0] -= F1
    for n in range(N - 1):
        Hd = model.hvp(R[n], d[n])
        G[n] += -K[:, None] * d[n] + 0.5 * Hd
        G[n + 1] += K[:, None] * d[n]
    u1 = model.energy(R[0])
    es = float(np.sum(0.5 * K[None, :, None] * d * d)) if d.size else 0.0
    return G, u1 + es


def fd_term(model, Rn, dn, h):
    """Finite-difference Hessian term of eq. (5):
    [F(R^n + eps d^n) - F(R^n - eps d^n)] / (4 eps), which tends to -1/2 H(R^n) d^n.
    eps is a pure number; it is set from a displacement length h as
    eps = h / max_i |d^n_i| so that no atom moves by more than h."""
    dmax = float(np.sqrt(np.max(np.sum(dn * dn, axis=1))))
    eps = h / dmax if dmax > 0 else 0.0
    if eps == 0.0:
        return np.zeros_like(dn), 0.0
    Fp = model.forces(Rn + eps * dn)
    Fm = model.forces(Rn - eps * dn)
    return (Fp - Fm) / (4.0 * eps), eps


def veff_grad_fd(model, R, h):
    """Gradient with the finite-difference term of eq. (5) in place of 1/2 H d:
    G^n = -[n=1] F^1 + [n>=2] K d^{n-1} + [n<=N-1] (-K d^n - D^n)."""
    R = np.asarray(R, np.float64)
    N = R.shape[0]
    _, K = coefficients(model)
    d, F = residuals(model, R)
    G = np.zeros_like(R)
    G[0] -= F[0] if N > 1 else model.forces(R[0])
    for n in range(N - 1):
        D, _ = fd_term(model, R[n], d[n], h)
        G[n] += -K[:, None] * d[n] - D
        G[n + 1] += K[:, None] * d[n]
    return G


def effective_forces_literal(model, R, eps):
    """F_eff^n evaluated literally from eqs. (5), (6), (7), with L^n = c F^n,
    eta^n = R^{n+1} - R^n - L^n and a fixed finite-difference parameter eps.
    Differences of bead coordinates use the minimum image."""
    R = np.asarray(R, np.float64)
    N = R.shape[0]
    assert N >= 2
    c, K = coefficients(model)
    Kc = K[:, None]
    F = [model.forces(R[n]) for n in range(N)]
    box = model.box

    def fd(n):
        eta = min_image(R[n + 1] - R[n], box) - c[:, None] * F[n]
        return (model.forces(R[n] + eps * eta) - model.forces(R[n] - eps * eta)) / (4.0 * eps)

    out = np.zeros_like(R)
    # eq. (6): first bead
    out[0] = 0.5 * F[0] + Kc * min_image(R[1] - R[0], box) + fd(0)
    # eq. (5): interior beads, 2 R^n - R^{n-1} - R^{n+1} written with minimum images
    for n in range(1, N - 1):
        two_r = min_image(R[n] - R[n - 1], box) - min_image(R[n + 1] - R[n], box)
        out[n] = -Kc * two_r + 0.5 * (F[n - 1] - F[n]) + fd(n)
    # eq. (7): last bead
    out[N - 1] = -Kc * min_image(R[N - 1] - R[N - 2], box) + 0.5 * F[N - 2]
    return out
