"""Short-range potential, force and Hessian-vector product -- FP64 brute force.

TEST INFRASTRUCTURE ONLY (see the package docstring): no product code imports this.

The paper's physical system (section 1.1) is Q atoms in a periodic box with potential
U(R) and force F = -grad U (eq. 1).  The paper's benchmark force field is not shipped;
the potential here is the short-range part of such a force field, each term written
out from its textbook definition:

  U = sum_{i<j, r_ij < r_c, (i,j) not excluded} [phi_LJ(r_ij) + phi_RF(r_ij)]_sf
      + sum_bonds k_b/2 (r - r0)^2

  phi_LJ(r) = c12/r^12 - c6/r^6, c6 = 4 eps sig^6, c12 = 4 eps sig^12,
              Lorentz-Berthelot mixing sig_ij = (sig_i + sig_j)/2, eps_ij = sqrt(eps_i eps_j)
  phi_RF(r) = (f/eps_r) q_i q_j (1/r + k_rf r^2 - c_rf),
              k_rf = (eps_rf - eps_r) / ((2 eps_rf + eps_r) r_c^3), c_rf = 1/r_c + k_rf r_c^2
  [phi]_sf(r) = phi(r) - phi(r_c) - (r - r_c) phi'(r_c)     (shifted force: phi and phi'
              both vanish at the cutoff, so forces are continuous and finite
              differences of forces converge)

Excluded pairs: atoms one or two bonds apart (1-2 and 1-3 neighbours in the bond
graph), from both LJ and RF.

Particle-mesh Ewald electrostatics (system key elec = "pme"; the paper's own runs use
PME, Appendix A.1) replaces phi_RF by the Ewald real-space term and adds the
reciprocal, self, background and excluded-pair terms (ewald.py, pme.py):

  phi_real(r) = f q_i q_j erfc(beta r)/r, shifted-force at r_c like the other pair terms
              (erfc(beta r_c) = ewald_rtol fixes beta)
  excluded pairs within r_c:  -f q_i q_j erf(beta r)/r   (no cut-off modifier)
  + E_rec (smooth PME, order pme_order, grid pme_grid) - f beta/sqrt(pi) sum q^2
  - f pi (sum q)^2 / (2 V beta^2)

Derivatives, for a pair with separation vector d = x_j - x_i and r = |d|:
  g = phi'(r)/r,   h = (phi''(r) - phi'(r)/r)/r^2
  F_i += g d,  F_j -= g d                                   (F = -grad U)
  (H v)_i += g (v_i - v_j) + h (d . (v_i - v_j)) d,  (H v)_j -= the same
(the 3x3 block of the pair Hessian is g I + h d d^T; it is even in d).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf as _np_erf
from scipy.special import erfc as _np_erfc

F_ELEC = 138.935458  # kJ mol^-1 nm e^-2, electric conversion factor 1/(4 pi eps0)


def reaction_field_constants(rc, eps_rf, eps_r=1.0):
    """k_rf and c_rf of the reaction-field pair potential (k_rf sets the dielectric
    continuum beyond r_c; c_rf makes phi_RF(r_c) = 0)."""
    krf = (eps_rf - eps_r) / ((2.0 * eps_rf + eps_r) * rc ** 3)
    crf = 1.0 / rc + krf * rc ** 2
    return krf, crf


# --- pair terms: phi, phi', phi'' (plain arithmetic: works on numpy arrays and on torch
# --- tensors, so the test suite can differentiate the same energy automatically)

def lj_phi(r, c6, c12):
    return c12 / r ** 12 - c6 / r ** 6


def lj_d1(r, c6, c12):
    return -12.0 * c12 / r ** 13 + 6.0 * c6 / r ** 7


def lj_d2(r, c6, c12):
    return 156.0 * c12 / r ** 14 - 42.0 * c6 / r ** 8


def rf_phi(r, qq, krf, crf):
    return qq * (1.0 / r + krf * r ** 2 - crf)


def rf_d1(r, qq, krf, crf):
    return qq * (-1.0 / r ** 2 + 2.0 * krf * r)


def rf_d2(r, qq, krf, crf):
    return qq * (2.0 / r ** 3 + 2.0 * krf)


def _erfc(x):
    if isinstance(x, np.ndarray) or np.isscalar(x):
        return _np_erfc(x)
    import torch
    return torch.special.erfc(x)


def _exp(x):
    if isinstance(x, np.ndarray) or np.isscalar(x):
        return np.exp(x)
    import torch
    return torch.exp(x)


def ewald_phi(r, qq, beta):
    """Ewald real-space pair energy qq erfc(beta r)/r."""
    return qq * _erfc(beta * r) / r


def ewald_d1(r, qq, beta):
    D = 2.0 * beta / math.sqrt(math.pi) * _exp(-(beta * r) ** 2)
    return qq * (-_erfc(beta * r) / r ** 2 - D / r)


def ewald_d2(r, qq, beta):
    D = 2.0 * beta / math.sqrt(math.pi) * _exp(-(beta * r) ** 2)
    return qq * (2.0 * _erfc(beta * r) / r ** 3 + D * (2.0 / r ** 2 + 2.0 * beta ** 2))


def excl_phi(r, qq, beta):
    """Excluded-pair correction -qq erf(beta r)/r = qq (erfc(beta r) - 1)/r."""
    return qq * (_erfc(beta * r) - 1.0) / r


def excl_d1(r, qq, beta):
    D = 2.0 * beta / math.sqrt(math.pi) * _exp(-(beta * r) ** 2)
    return qq * (-(_erfc(beta * r) - 1.0) / r ** 2 - D / r)


def excl_d2(r, qq, beta):
    D = 2.0 * beta / math.sqrt(math.pi) * _exp(-(beta * r) ** 2)
    return qq * (2.0 * (_erfc(beta * r) - 1.0) / r ** 3 + D * (2.0 / r ** 2 + 2.0 * beta ** 2))


def bond_phi(r, r0, kb):
    return 0.5 * kb * (r - r0) ** 2


def bond_d1(r, r0, kb):
    return kb * (r - r0)


def bond_d2(r, r0, kb):
    return kb + 0.0 * r


def min_image(d, box):
    """Minimum-image convention in an orthorhombic periodic box."""
    return d - box * np.rint(d / box)


class Model:
    """Force-field constants of one system, derived only from the system description."""

    def __init__(self, system):
        s = system
        self.Q = int(s["Q"])
        self.box = np.asarray(s["box"], np.float64)
        self.rc = float(s["rc"])
        if not self.rc < 0.5 * self.box.min():
            raise ValueError("cutoff must be below half the smallest box length")
        self.type = np.asarray(s["type"], np.int64)
        sig = np.asarray(s["sigma"], np.float64)
        eps = np.asarray(s["epsilon"], np.float64)
        sij = 0.5 * (sig[:, None] + sig[None, :])
        eij = np.sqrt(eps[:, None] * eps[None, :])
        self.c6 = 4.0 * eij * sij ** 6
        self.c12 = 4.0 * eij * sij ** 12
        self.eps_r = float(s.get("eps_r", 1.0))
        self.krf, self.crf = reaction_field_constants(self.rc, float(s["eps_rf"]), self.eps_r)
        self.q = np.asarray(s["charge"], np.float64)
        self.fq = F_ELEC / self.eps_r
        self.bonds = np.asarray(s["bonds"], np.int64).reshape(-1, 2)
        self.bond_r0 = np.asarray(s["bond_r0"], np.float64)
        self.bond_k = np.asarray(s["bond_k"], np.float64)
        self.mass = np.asarray(s["mass"], np.float64)
        self.dt, self.nu = float(s["dt"], ), float(s["nu"])
        self.excluded = self._exclusions()
        self.elec = str(s.get("elec", "rf"))
        if self.elec not in ("rf", "pme"):
            raise ValueError("elec must be 'rf' or 'pme'")
        self.pme = None
        if self.elec == "pme":
            from . import ewald
            from .pme import PME
            self.beta = ewald.beta_from_rtol(self.rc, float(s.get("ewald_rtol", 1e-5)))
            self.pme = PME(self.box, s["pme_grid"], int(s.get("pme_order", 4)), self.beta,
                           self.q, self.fq)
            V = float(np.prod(self.box))
            self.e_const = (-self.fq * self.beta / math.sqrt(math.pi) * float(np.sum(self.q ** 2))
                            - self.fq * math.pi * float(np.sum(self.q)) ** 2
                            / (2.0 * V * self.beta ** 2))

    def _exclusions(self):
        """Sorted codes i*Q + j (i < j) of pairs one or two bonds apart."""
        Q = self.Q
        nbr = [set() for _ in range(Q)]
        for i, j in self.bonds:
            nbr[i].add(int(j))
            nbr[j].add(int(i))
        codes = set()
        for i in range(Q):
            for j in nbr[i]:
                codes.add((min(i, j), max(i, j)))
                for k in nbr[j]:
                    if k != i:
                        codes.add((min(i, k), max(i, k)))
        if not codes:
            return np.zeros(0, np.int64)
        a = np.array(sorted(codes), np.int64)
        return np.sort(a[:, 0] * Q + a[:, 1])

    # -- pair set -------------------------------------------------------------------
    def pairs(self, X, block=512):
        """All non-excluded pairs i < j with minimum-image distance below r_c.
        Returns (i, j, d) with d = x_j - x_i (minimum image)."""
        X = np.asarray(X, np.float64)
        Q = self.Q
        rc2 = self.rc ** 2
        I, J, D = [], [], []
        jj = np.arange(Q)
        for i0 in range(0, Q, block):
            i1 = min(Q, i0 + block)
            d = X[None, :, :] - X[i0:i1, None, :]
            d = min_image(d, self.box)
            r2 = np.einsum("abk,abk->ab", d, d)
            m = (jj[None, :] > np.arange(i0, i1)[:, None]) & (r2 < rc2)
            a, b = np.nonzero(m)
            I.append(a + i0)
            J.append(b)
            D.append(d[a, b])
        i = np.concatenate(I)
        j = np.concatenate(J)
        d = np.concatenate(D) if D else np.zeros((0, 3))
        if self.excluded.size:
            keep = ~np.isin(i * Q + j, self.excluded)
            i, j, d = i[keep], j[keep], d[keep]
        return i, j, d

    # -- pair energy and derivatives --------------------------------------------------
    def pair_phi(self, r, i, j):
        """Shifted-force pair energy (LJ + RF) for pairs (i, j) at distance r.
        r may also be a torch tensor (constants are converted to match)."""
        ti, tj = self.type[i], self.type[j]
        c6, c12 = self.c6[ti, tj], self.c12[ti, tj]
        qq = self.fq * self.q[i] * self.q[j]
        if not isinstance(r, np.ndarray):
            c6, c12, qq = r.new_tensor(c6), r.new_tensor(c12), r.new_tensor(qq)
        rc = self.rc
        phi = lj_phi(r, c6, c12) + self._el_phi(r, qq)
        phic = lj_phi(rc, c6, c12) + self._el_phi(rc, qq)
        d1c = lj_d1(rc, c6, c12) + self._el_d1(rc, qq)
        return phi - phic - (r - rc) * d1c

    def _el_phi(self, r, qq):
        if self.elec == "pme":
            return ewald_phi(r, qq, self.beta)
        return rf_phi(r, qq, self.krf, self.crf)

    def _el_d1(self, r, qq):
        if self.elec == "pme":
            return ewald_d1(r, qq, self.beta)
        return rf_d1(r, qq, self.krf, self.crf)

    def _el_d2(self, r, qq):
        if self.elec == "pme":
            return ewald_d2(r, qq, self.beta)
        return rf_d2(r, qq, self.krf, self.crf)

    def pair_gh(self, r, i, j):
        """g = phi_sf'/r and h = (phi'' - phi_sf'/r)/r^2 for pairs (i, j)."""
        ti, tj = self.type[i], self.type[j]
        c6, c12 = self.c6[ti, tj], self.c12[ti, tj]
        qq = self.fq * self.q[i] * self.q[j]
        rc = self.rc
        d1 = lj_d1(r, c6, c12) + self._el_d1(r, qq)
        d1 = d1 - (lj_d1(rc, c6, c12) + self._el_d1(rc, qq))
        d2 = lj_d2(r, c6, c12) + self._el_d2(r, qq)
        g = d1 / r
        h = (d2 - g) / r ** 2
        return g, h

    # -- PME: excluded pairs within the cut-off carry -f q_i q_j erf(beta r)/r ----------
    def excluded_pairs(self, X):
        """Excluded pairs (i < j) within r_c: (i, j, d), d = x_j - x_i (minimum image)."""
        if not self.excluded.size:
            z = np.zeros(0, np.int64)
            return z, z, np.zeros((0, 3))
        i = self.excluded // self.Q
        j = self.excluded % self.Q
        d = min_image(np.asarray(X, np.float64)[j] - np.asarray(X, np.float64)[i], self.box)
        r2 = np.einsum("ak,ak->a", d, d)
        keep = r2 < self.rc ** 2
        return i[keep], j[keep], d[keep]

    def _excl_terms(self, X):
        i, j, d = self.excluded_pairs(X)
        r = np.sqrt(np.einsum("ak,ak->a", d, d))
        qq = self.fq * self.q[i] * self.q[j]
        d1 = excl_d1(r, qq, self.beta)
        g = d1 / r
        h = (excl_d2(r, qq, self.beta) - g) / r ** 2
        return i, j, d, r, qq, g, h

    def bond_vectors(self, X):
        b = self.bonds
        d = min_image(X[b[:, 1]] - X[b[:, 0]], self.box)
        return b[:, 0], b[:, 1], d

    # -- public: energy, force, Hessian-vector product --------------------------------
    def energy(self, X):
        """U(X) (kJ/mol)."""
        X = np.asarray(X, np.float64)
        i, j, d = self.pairs(X)
        r = np.sqrt(np.einsum("ak,ak->a", d, d))
        e = float(np.sum(self.pair_phi(r, i, j)))
        if len(self.bonds):
            bi, bj, bd = self.bond_vectors(X)
            br = np.sqrt(np.einsum("ak,ak->a", bd, bd))
            e += float(np.sum(bond_phi(br, self.bond_r0, self.bond_k)))
        if self.pme is not None:
            _, _, _, r, qq, _, _ = self._excl_terms(X)
            e += float(np.sum(excl_phi(r, qq, self.beta)))
            e += self.pme.energy(X) + self.e_const
        return e

    def forces(self, X):
        """F = -grad U (Q, 3)."""
        X = np.asarray(X, np.float64)
        F = np.zeros((self.Q, 3))
        i, j, d = self.pairs(X)
        r = np.sqrt(np.einsum("ak,ak->a", d, d))
        g, _ = self.pair_gh(r, i, j)
        f = g[:, None] * d
        np.add.at(F, i, f)
        np.add.at(F, j, -f)
        if len(self.bonds):
            bi, bj, bd = self.bond_vectors(X)
            br = np.sqrt(np.einsum("ak,ak->a", bd, bd))
            bg = bond_d1(br, self.bond_r0, self.bond_k) / br
            f = bg[:, None] * bd
            np.add.at(F, bi, f)
            np.add.at(F, bj, -f)
        if self.pme is not None:
            ei, ej, ed, _, _, eg, _ = self._excl_terms(X)
            f = eg[:, None] * ed
            np.add.at(F, ei, f)
            np.add.at(F, ej, -f)
            F += self.pme.forces(X)
        return F

    def hvp(self, X, V):
        """H(X) V with H the Hessian of U (Q, 3)."""
        X = np.asarray(X, np.float64)
        V = np.asarray(V, np.float64)
        out = np.zeros((self.Q, 3))
        i, j, d = self.pairs(X)
        r = np.sqrt(np.einsum("ak,ak->a", d, d))
        g, h = self.pair_gh(r, i, j)
        self._hvp_acc(out, i, j, d, g, h, V)
        if len(self.bonds):
            bi, bj, bd = self.bond_vectors(X)
            br = np.sqrt(np.einsum("ak,ak->a", bd, bd))
            d1 = bond_d1(br, self.bond_r0, self.bond_k)
            bg = d1 / br
            bh = (bond_d2(br, self.bond_r0, self.bond_k) - bg) / br ** 2
            self._hvp_acc(out, bi, bj, bd, bg, bh, V)
        if self.pme is not None:
            ei, ej, ed, _, _, eg, eh = self._excl_terms(X)
            self._hvp_acc(out, ei, ej, ed, eg, eh, V)
            out += self.pme.hvp(X, V)
        return out

    @staticmethod
    def _hvp_acc(out, i, j, d, g, h, V):
        dv = V[i] - V[j]
        s = np.einsum("ak,ak->a", d, dv)
        t = g[:, None] * dv + (h * s)[:, None] * d
        np.add.at(out, i, t)
        np.add.at(out, j, -t)
