"""Metadynamics of paths (section 1.2): the end-to-end collective variable of eq. (8) and
a Gaussian metadynamics bias on it (oracle side, plain FP64).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the benchmark's CPU
baseline, never by the library.

- Order parameter s(R): the distance between the centres of mass of two atom groups A and
  B (section 3 takes the ligand and the binding pocket).  In a periodic box each group's
  centre of mass is taken from its atoms' minimum-image offsets to the group's first atom
  (groups smaller than half the box), and the distance from the minimum image of the
  difference of the two centres.
- End-to-end variable (eq. 8): S = s(R^N) - s(R^1).
- Bias: V(S) = sum_k w_k exp(-(S - S_k)^2 / (2 sigma^2)) over the deposited Gaussians.
  A Gaussian is added at the current S every `stride` steps.  Standard metadynamics keeps
  w_k = w0; the well-tempered variant (bias factor gamma > 1) uses
  w_k = w0 exp(-V(S_k) / (kT (gamma - 1))).
- Its gradient reaches only beads 1 and N:
  dV/dR^N = V'(S) ds/dR^N,  dV/dR^1 = -V'(S) ds/dR^1,
  ds/dr_i = +(m_i / M_B) e for i in B and -(m_i / M_A) e for i in A, e = d / |d|.
"""
from __future__ import annotations

import numpy as np


def _mi(d, box):
    return d - box * np.rint(d / box)


def com(X, idx, mass, box):
    """Centre of mass of atoms idx of configuration X (Q, 3)."""
    idx = np.asarray(idx)
    ref = X[idx[0]]
    off = _mi(X[idx] - ref, box)
    m = mass[idx]
    return ref + (m[:, None] * off).sum(0) / m.sum()


def order_parameter(X, A, B, mass, box):
    """s(X) = |mi(COM_B - COM_A)| and the unit vector e along the difference."""
    d = _mi(com(X, B, mass, box) - com(X, A, mass, box), box)
    s = float(np.sqrt(np.dot(d, d)))
    return s, d / s


def ds_dx(X, A, B, mass, box):
    """Gradient of s with respect to every atom of X, (Q, 3)."""
    s, e = order_parameter(X, A, B, mass, box)
    g = np.zeros_like(X)
    A = np.asarray(A)
    B = np.asarray(B)
    g[A] -= (mass[A] / mass[A].sum())[:, None] * e
    g[B] += (mass[B] / mass[B].sum())[:, None] * e
    return g


def end_to_end(R, A, B, mass, box):
    """S of eq. (8) for a path R (N, Q, 3)."""
    return order_parameter(R[-1], A, B, mass, box)[0] - order_parameter(R[0], A, B, mass, box)[0]


def bias(S, centers, heights, sigma):
    """V(S) and dV/dS for Gaussians at `centers` with `heights`."""
    c = np.asarray(centers, np.float64)
    w = np.asarray(heights, np.float64)
    if c.size == 0:
        return 0.0, 0.0
    x = S - c
    g = w * np.exp(-0.5 * x * x / (sigma * sigma))
    return float(g.sum()), float((-x / (sigma * sigma) * g).sum())


def bias_gradient(R, A, B, mass, box, centers, heights, sigma):
    """(S, V(S), gradient of V with respect to the path, (N, Q, 3))."""
    S = end_to_end(R, A, B, mass, box)
    V, dV = bias(S, centers, heights, sigma)
    G = np.zeros_like(R)
    G[-1] += dV * ds_dx(R[-1], A, B, mass, box)
    G[0] -= dV * ds_dx(R[0], A, B, mass, box)
    return S, V, G


def new_height(S, centers, heights, sigma, height0, bias_factor, kT):
    """Height of a Gaussian deposited at S: w0, or w0 exp(-V(S) / (kT (gamma - 1)))."""
    if bias_factor and bias_factor > 1.0:
        V, _ = bias(S, centers, heights, sigma)
        return height0 * np.exp(-V / (kT * (bias_factor - 1.0)))
    return height0


class Bias:
    """Deposition state of one metadynamics run on the end-to-end variable."""

    def __init__(self, A, B, mass, box, sigma, height, bias_factor=0.0, kT=0.0, stride=1):
        self.A = np.asarray(A)
        self.B = np.asarray(B)
        self.mass = np.asarray(mass, np.float64)
        self.box = np.asarray(box, np.float64)
        self.sigma = float(sigma)
        self.height = float(height)
        self.bias_factor = float(bias_factor)
        self.kT = float(kT)
        self.stride = int(stride)
        self.centers = []
        self.heights = []

    def apply(self, R, step=None):
        """(S, V(S), gradient) with the Gaussians deposited so far; then, when `step` is
        a multiple of the stride, deposit a Gaussian at S."""
        S, V, G = bias_gradient(R, self.A, self.B, self.mass, self.box, self.centers,
                                self.heights, self.sigma)
        if step is not None and step % self.stride == 0:
            self.heights.append(new_height(S, self.centers, self.heights, self.sigma,
                                           self.height, self.bias_factor, self.kT))
            self.centers.append(S)
        return S, V, G
