"""Smooth particle-mesh Ewald (reciprocal part) with its forces and exact Hessian-vector
product -- FP64, TEST INFRASTRUCTURE ONLY.

The paper's standard MD runs (Appendix A.1) use particle-mesh Ewald for long-range
electrostatics.  The method is the smooth PME of Essmann et al. (J. Chem. Phys. 103,
8577, 1995); its steps are written out here in that paper's order and notation:

  1. scaled fractional coordinates u_ia = K_a frac(x_ia / L_a) on a K_x x K_y x K_z grid;
  2. the charge grid  Q(k) = sum_i q_i M_p(u_ix - k_x) M_p(u_iy - k_y) M_p(u_iz - k_z),
     periodic in k, with M_p the cardinal B-spline of order p;
  3. the influence function B(m) C(m),
        C(m) = exp(-pi^2 |m|^2 / beta^2) / (pi V |m|^2)  (m != 0),  C(0) = 0,
        B(m) = prod_a |b_a(m_a)|^2,
        |b_a(m)|^2 = 1 / |sum_{k=0}^{p-2} M_p(k + 1) exp(2 pi i m k / K_a)|^2,
     with m = (m_x/L_x, m_y/L_y, m_z/L_z), m_a the signed DFT frequency;
  4. phi = DFT^-1 [f B C DFT[Q]] (the unnormalised inverse transform, so that phi is
     the grid potential of the convolution), and E_rec = 1/2 sum_k Q(k) phi(k);
  5. forces F_i = -q_i sum_k grad theta_i(k) phi(k), theta_i(k) the product of the three
     spline weights of atom i at grid point k.

The Hessian-vector product is the directional derivative of the forces, written out
for the quadratic form E = 1/2 Q^T A Q (A the symmetric convolution of step 4):

  (H v)_i = q_i sum_k grad theta_i(k) . dphi(k) + q_i sum_k [grad grad theta_i(k) v_i] phi(k),
  dphi = DFT^-1 [f B C DFT[dQ]],  dQ(k) = sum_j q_j grad theta_j(k) . v_j,

i.e. the grid of "dipoles" q_j v_j is spread with the gradient of the spline weights,
convolved like the charges, and gathered back with the gradient; the second term
comes from the curvature of the spline weights themselves.

Reading: orders p are even (4, 6, 8).  For odd p the sum in |b(m)|^2 vanishes at the
Nyquist frequency; even orders avoid that, and p >= 4 keeps the weights twice
differentiable, which the Hessian needs.
"""
from __future__ import annotations

import numpy as np


def cardinal_bspline(n, x):
    """M_n(x): M_2(x) = 1 - |x - 1| on [0, 2] (0 elsewhere) and the recursion
    M_n(x) = [x M_{n-1}(x) + (n - x) M_{n-1}(x - 1)] / (n - 1)."""
    x = np.asarray(x, np.float64)
    if n == 2:
        return np.where((x >= 0.0) & (x <= 2.0), 1.0 - np.abs(x - 1.0), 0.0)
    return (x * cardinal_bspline(n - 1, x) + (n - x) * cardinal_bspline(n - 1, x - 1.0)) / (n - 1)


def cardinal_bspline_d1(n, x):
    """dM_n/dx = M_{n-1}(x) - M_{n-1}(x - 1)."""
    return cardinal_bspline(n - 1, x) - cardinal_bspline(n - 1, np.asarray(x) - 1.0)


def cardinal_bspline_d2(n, x):
    """d^2 M_n/dx^2 = M_{n-2}(x) - 2 M_{n-2}(x - 1) + M_{n-2}(x - 2)."""
    x = np.asarray(x, np.float64)
    return (cardinal_bspline(n - 2, x) - 2.0 * cardinal_bspline(n - 2, x - 1.0)
            + cardinal_bspline(n - 2, x - 2.0))


def bspline_moduli(p, K):
    """|b(m)|^2 for m = 0 .. K-1 (DFT order)."""
    k = np.arange(p - 1)
    Mk = cardinal_bspline(p, k + 1.0)
    m = np.arange(K)
    den = np.exp(2j * np.pi * np.outer(m, k) / K) @ Mk
    return 1.0 / np.abs(den) ** 2


class PME:
    """Reciprocal-space PME energy, forces and Hessian-vector product of one system.

    box (3,), grid (K_x, K_y, K_z), order p (even, >= 4), beta (nm^-1), charges q (e),
    f the Coulomb factor (kJ mol^-1 nm e^-2, already divided by eps_r).
    """

    def __init__(self, box, grid, order, beta, q, f):
        self.box = np.asarray(box, np.float64)
        self.K = np.asarray(grid, np.int64)
        self.p = int(order)
        if self.p < 4 or self.p % 2:
            raise ValueError("PME order must be even and at least 4")
        if np.any(self.K < self.p):
            raise ValueError("PME grid must have at least `order` points per axis")
        self.beta = float(beta)
        self.q = np.asarray(q, np.float64)
        self.f = float(f)
        self.phihat = self.influence()

    def influence(self):
        """f B(m) C(m) on the full DFT grid."""
        V = float(np.prod(self.box))
        ms = [np.fft.fftfreq(int(K), d=1.0 / int(K)) / L for K, L in zip(self.K, self.box)]
        mx, my, mz = np.meshgrid(*ms, indexing="ij")
        m2 = mx ** 2 + my ** 2 + mz ** 2
        with np.errstate(divide="ignore", invalid="ignore"):
            C = np.exp(-np.pi ** 2 * m2 / self.beta ** 2) / (np.pi * V * m2)
        C[0, 0, 0] = 0.0
        b = [bspline_moduli(self.p, int(K)) for K in self.K]
        B = b[0][:, None, None] * b[1][None, :, None] * b[2][None, None, :]
        return self.f * B * C

    # -- spline weights ------------------------------------------------------------
    def weights(self, X):
        """Per atom and axis: grid indices (Q, 3, p), weights, first and second
        derivatives with respect to the Cartesian coordinate (chain rule du/dx = K/L)."""
        X = np.asarray(X, np.float64)
        s = X / self.box
        u = self.K * (s - np.floor(s))
        base = np.floor(u)
        w = u - base
        j = np.arange(self.p)
        x = w[:, :, None] + j                                  # (Q, 3, p): u - k
        idx = np.mod(base.astype(np.int64)[:, :, None] - j, self.K[None, :, None])
        kl = (self.K / self.box)[None, :, None]
        th = cardinal_bspline(self.p, x)
        dth = cardinal_bspline_d1(self.p, x) * kl
        d2th = cardinal_bspline_d2(self.p, x) * kl ** 2
        return idx, th, dth, d2th

    def _spread(self, idx, wq):
        """Grid with wq[i, a, b, c] added at (idx[i,0,a], idx[i,1,b], idx[i,2,c])."""
        G = np.zeros(tuple(int(K) for K in self.K))
        ix = idx[:, 0, :, None, None]
        iy = idx[:, 1, None, :, None]
        iz = idx[:, 2, None, None, :]
        np.add.at(G, (np.broadcast_to(ix, wq.shape), np.broadcast_to(iy, wq.shape),
                      np.broadcast_to(iz, wq.shape)), wq)
        return G

    def _gather(self, idx, G):
        """G at every (atom, a, b, c) spline point: (Q, p, p, p)."""
        return G[idx[:, 0, :, None, None], idx[:, 1, None, :, None], idx[:, 2, None, None, :]]

    def convolve(self, G):
        """DFT^-1 [f B C DFT[G]] with the unnormalised inverse transform."""
        return np.real(np.fft.ifftn(self.phihat * np.fft.fftn(G))) * float(np.prod(self.K))

    def charge_grid(self, X):
        idx, th, _, _ = self.weights(X)
        wq = self.q[:, None, None, None] * (th[:, 0, :, None, None] * th[:, 1, None, :, None]
                                            * th[:, 2, None, None, :])
        return self._spread(idx, wq)

    # -- energy, forces, Hessian-vector product -------------------------------------
    def energy(self, X):
        Qg = self.charge_grid(X)
        return 0.5 * float(np.sum(Qg * self.convolve(Qg)))

    @staticmethod
    def _grad_theta(th, dth):
        """grad theta_i(k) as (Q, 3, p, p, p)."""
        tx, ty, tz = th[:, 0, :, None, None], th[:, 1, None, :, None], th[:, 2, None, None, :]
        dx, dy, dz = dth[:, 0, :, None, None], dth[:, 1, None, :, None], dth[:, 2, None, None, :]
        return np.stack([dx * ty * tz, tx * dy * tz, tx * ty * dz], 1)

    def forces(self, X):
        idx, th, dth, _ = self.weights(X)
        Qg = self._spread(idx, self.q[:, None, None, None] * (
            th[:, 0, :, None, None] * th[:, 1, None, :, None] * th[:, 2, None, None, :]))
        phi = self.convolve(Qg)
        gt = self._grad_theta(th, dth)
        ph = self._gather(idx, phi)
        return -self.q[:, None] * np.einsum("iaxyz,ixyz->ia", gt, ph)

    def hvp(self, X, V):
        """H_rec(X) V (Q, 3)."""
        V = np.asarray(V, np.float64)
        idx, th, dth, d2th = self.weights(X)
        tx, ty, tz = th[:, 0, :, None, None], th[:, 1, None, :, None], th[:, 2, None, None, :]
        dx, dy, dz = dth[:, 0, :, None, None], dth[:, 1, None, :, None], dth[:, 2, None, None, :]
        hx, hy, hz = d2th[:, 0, :, None, None], d2th[:, 1, None, :, None], d2th[:, 2, None, None, :]
        Qg = self._spread(idx, self.q[:, None, None, None] * (tx * ty * tz))
        phi = self.convolve(Qg)
        gt = np.stack([dx * ty * tz, tx * dy * tz, tx * ty * dz], 1)       # (Q, 3, p, p, p)
        dQ = self._spread(idx, self.q[:, None, None, None] * np.einsum("iaxyz,ia->ixyz", gt, V))
        dphi = self.convolve(dQ)
        # grad grad theta (Q, 3, 3, p, p, p)
        hh = np.empty((len(V), 3, 3) + gt.shape[2:])
        hh[:, 0, 0] = hx * ty * tz
        hh[:, 1, 1] = tx * hy * tz
        hh[:, 2, 2] = tx * ty * hz
        hh[:, 0, 1] = hh[:, 1, 0] = dx * dy * tz
        hh[:, 0, 2] = hh[:, 2, 0] = dx * ty * dz
        hh[:, 1, 2] = hh[:, 2, 1] = tx * dy * dz
        ph = self._gather(idx, phi)
        dph = self._gather(idx, dphi)
        t1 = np.einsum("iaxyz,ixyz->ia", gt, dph)
        t2 = np.einsum("iabxyz,ib,ixyz->ia", hh, V, ph)
        return self.q[:, None] * (t1 + t2)
