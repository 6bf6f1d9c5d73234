"""Path molecular dynamics (eq. 4) on V_eff: the oracle's integrator, plain FP64.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the benchmark's CPU
baseline, never by the library.

Section 1.1 evolves the whole polymer (every bead n = 1..N) by Newton's equations
M R''^n = F^n_eff = -grad_{R^n} V_eff (eq. 4), with a thermostat for sampling at
temperature T (eq. 2: p ~ exp(-V_eff / kT)).  Appendix A.2 uses velocity Verlet for
constant energy and a Langevin thermostat for constant temperature.  Here both are one
splitting, B A O A B (Leimkuhler and Matthews, 2013), with step tau:

    B: V <- V - tau/2 G / M            (G = grad V_eff at the current R)
    A: R <- R + tau/2 V
    O: V <- c1 V + c2 xi / sqrt(M),    c1 = exp(-gamma tau), c2 = sqrt((1 - c1^2) kT)
    A: R <- R + tau/2 V
       G <- grad V_eff(R)
    B: V <- V - tau/2 G / M

gamma = 0 drops O and leaves velocity Verlet.  xi are the counter-based deviates of
`oracle.philox.path_normals`.  The fictitious masses M of eq. (4) are not fixed by the
paper; they are read as the atoms' physical masses, the same for every bead.

With a metadynamics bias on the end-to-end variable of eq. (8) (`oracle.mop_bias.Bias`),
the gradient of each step adds the bias gradient computed with the Gaussians deposited so
far; then, at steps that are multiples of the deposition stride, a Gaussian is added at
the current value of the variable.
"""
from __future__ import annotations

import numpy as np

from . import path as OP
from .philox import path_normals


def kinetic(M, V):
    """sum_n sum_i M_i/2 |V^n_i|^2."""
    return float(0.5 * np.sum(M[None, :, None] * V * V))


def baoab_step(model, R, V, G, M, tau, gamma=0.0, kT=0.0, seed=0, step=0, bias=None):
    """One step.  R, V, G: [N][Q][3]; G must be the gradient of the total potential at R
    (V_eff, plus the bias when `bias` is an `oracle.mop_bias.Bias`).  Returns the new
    (R, V, G, V_eff, kinetic energy, V_bias, S)."""
    R = np.array(R, np.float64, copy=True)
    V = np.array(V, np.float64, copy=True)
    N, Q, _ = R.shape
    minv = 1.0 / np.asarray(M, np.float64)[None, :, None]
    V -= 0.5 * tau * G * minv
    R += 0.5 * tau * V
    if gamma > 0.0:
        c1 = np.exp(-gamma * tau)
        c2 = np.sqrt((1.0 - c1 * c1) * kT)
        V = c1 * V + c2 * np.sqrt(minv) * path_normals(seed, step, N, Q)
    R += 0.5 * tau * V
    G, veff = OP.veff_grad(model, R)
    S = vb = 0.0
    if bias is not None:
        S, vb, Gb = bias.apply(R, step)
        G = G + Gb
    V -= 0.5 * tau * G * minv
    return R, V, G, float(veff), kinetic(M, V), float(vb), float(S)


def run(model, R, V, M, tau, nsteps, gamma=0.0, kT=0.0, seed=0, step0=0, bias=None):
    """nsteps steps from (R, V); returns R, V, G and the per-step
    (V_eff, kinetic, V_bias, S)."""
    G, _ = OP.veff_grad(model, R)
    if bias is not None:
        G = G + bias.apply(R)[2]
    E = np.zeros((nsteps, 4))
    for k in range(nsteps):
        R, V, G, ve, ke, vb, S = baoab_step(model, R, V, G, M, tau, gamma, kT, seed, step0 + k,
                                            bias)
        E[k] = ve, ke, vb, S
    return R, V, G, E
