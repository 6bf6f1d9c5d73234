"""Pins of the oracle's Ewald / particle-mesh Ewald electrostatics (oracle/ewald.py,
oracle/pme.py and the elec = "pme" branch of oracle/potential.py).

- Cardinal B-splines: partition of unity, textbook values of M_4 at the integers,
  symmetry, derivatives against finite differences, |b(0)|^2 = 1.
- Ewald sum: the Madelung constants of rock salt and caesium chloride, independence of
  the splitting parameter, and the identity that excluding a pair removes exactly its
  bare Coulomb term.  Reciprocal forces against finite differences of the lattice sum.
- Smooth PME: energy and forces converge to the Ewald reciprocal sum as the order and
  the grid grow; forces are minus the finite-difference gradient of the PME energy; the
  Hessian-vector product is the finite-difference derivative of the forces and is
  symmetric.
- The full model with PME: total electrostatic energy equals the Ewald sum (tight
  splitting, fine grid); forces and Hessian-vector products against finite differences
  with LJ, bonds and excluded pairs; the real-space pair term reduces to bare Coulomb as
  beta -> 0.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import ewald as EW
from oracle import pme as PM
from oracle import potential as P
from oracle.potential import Model

F = P.F_ELEC


def _random_system(seed, Q=20, box=(1.8, 2.0, 2.2)):
    rng = np.random.default_rng(seed)
    box = np.asarray(box)
    X = rng.uniform(0.0, 1.0, (Q, 3)) * box
    q = rng.normal(0.0, 0.5, Q)
    return X, q - q.mean(), box


@pytest.mark.parametrize("p", [4, 6, 8])
def test_bspline_identities(p):
    w = np.linspace(0.0, 0.999, 37)
    x = w[:, None] + np.arange(p)
    assert np.allclose(PM.cardinal_bspline(p, x).sum(1), 1.0, atol=1e-14)
    assert np.allclose(PM.cardinal_bspline_d1(p, x).sum(1), 0.0, atol=1e-13)
    assert np.allclose(PM.cardinal_bspline_d2(p, x).sum(1), 0.0, atol=1e-12)
    y = np.linspace(0.05, p - 0.05, 41)
    assert np.allclose(PM.cardinal_bspline(p, y), PM.cardinal_bspline(p, p - y), atol=1e-15)
    h = 1e-5
    fd1 = (PM.cardinal_bspline(p, y + h) - PM.cardinal_bspline(p, y - h)) / (2 * h)
    fd2 = (PM.cardinal_bspline_d1(p, y + h) - PM.cardinal_bspline_d1(p, y - h)) / (2 * h)
    assert np.allclose(PM.cardinal_bspline_d1(p, y), fd1, atol=1e-9)
    assert np.allclose(PM.cardinal_bspline_d2(p, y), fd2, atol=1e-8)
    assert PM.bspline_moduli(p, 16)[0] == pytest.approx(1.0, rel=1e-14)


def test_cubic_bspline_textbook_values():
    M = PM.cardinal_bspline(4, np.array([0.0, 1.0, 2.0, 3.0, 4.0, 0.5]))
    assert np.allclose(M, [0.0, 1 / 6, 2 / 3, 1 / 6, 0.0, 1 / 48], atol=1e-15)


def _ewald_total(X, q, box, rc, rtol=1e-14, excluded=()):
    beta = EW.beta_from_rtol(rc, rtol)
    return EW.ewald_energy(X, q, box, beta, rc, F, excluded)["total"]


def test_madelung_constants():
    a = 0.5640
    fcc = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    X = np.concatenate([fcc, fcc + [0.5, 0, 0]]) * a
    q = np.array([1.0] * 4 + [-1.0] * 4)
    E = _ewald_total(X, q, np.full(3, a), 0.49 * a)
    M_nacl = -E * (a / 2) / (4 * F)
    assert M_nacl == pytest.approx(1.747564594633182, rel=1e-10)
    X = np.array([[0, 0, 0], [.5, .5, .5]]) * a
    E = _ewald_total(X, np.array([1.0, -1.0]), np.full(3, a), 0.49 * a)
    M_cscl = -E * (math.sqrt(3) * a / 2) / F
    assert M_cscl == pytest.approx(1.762674773070, rel=1e-10)


def test_ewald_independent_of_beta():
    X, q, box = _random_system(2)
    E = [_ewald_total(X, q, box, rc, rtol) for rc, rtol in
         [(0.6, 1e-12), (0.8, 1e-12), (0.85, 1e-14)]]
    assert np.ptp(E) < 1e-9 * abs(E[0])


def test_excluding_a_pair_removes_its_bare_coulomb_term():
    X, q, box = _random_system(3)
    d = P.min_image(X - X[2], box)
    dist = np.sqrt(np.einsum("ak,ak->a", d, d))
    dist[2] = np.inf
    j = int(np.argmin(dist))                       # the nearest partner of atom 2
    r = float(dist[j])
    assert r < 0.8
    beta = EW.beta_from_rtol(0.8, 1e-8)
    full = EW.ewald_energy(X, q, box, beta, 0.8, F)["total"]
    excl = EW.ewald_energy(X, q, box, beta, 0.8, F, excluded=[(j, 2)])["total"]
    assert excl == pytest.approx(full - F * q[2] * q[j] / r, rel=1e-12, abs=1e-10)


def test_ewald_recip_forces_against_fd():
    X, q, box = _random_system(4, Q=8)
    beta = 3.0
    Fr = EW.recip_forces(X, q, box, beta, F)
    h = 1e-6
    for i, a in [(0, 0), (3, 1), (7, 2)]:
        Xp, Xm = X.copy(), X.copy()
        Xp[i, a] += h
        Xm[i, a] -= h
        fd = -(EW.recip_energy(Xp, q, box, beta, F) - EW.recip_energy(Xm, q, box, beta, F)) / (2 * h)
        assert Fr[i, a] == pytest.approx(fd, rel=1e-7, abs=1e-7)


def test_pme_converges_to_ewald():
    X, q, box = _random_system(1, Q=30)
    beta = EW.beta_from_rtol(0.8, 1e-5)
    er = EW.recip_energy(X, q, box, beta, F)
    fr = EW.recip_forces(X, q, box, beta, F)
    errs = []
    for p, h in [(4, 0.12), (4, 0.06), (8, 0.06)]:
        K = [int(np.ceil(L / h)) for L in box]
        pm = PM.PME(box, K, p, beta, q, F)
        errs.append((abs(pm.energy(X) - er) / abs(er),
                     np.linalg.norm(pm.forces(X) - fr) / np.linalg.norm(fr)))
    assert errs[0][0] < 3e-3 and errs[1][0] < 2e-4 and errs[2][0] < 1e-7
    assert errs[0][1] < 3e-2 and errs[2][1] < 1e-5
    assert errs[0][0] > errs[1][0] > errs[2][0]


def test_pme_forces_and_hvp_against_fd():
    X, q, box = _random_system(5, Q=16)
    pm = PM.PME(box, [16, 18, 20], 4, 3.5, q, F)
    Fp = pm.forces(X)
    h = 1e-6
    fd = np.zeros_like(X)
    for i in range(len(q)):
        for a in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[i, a] += h
            Xm[i, a] -= h
            fd[i, a] = -(pm.energy(Xp) - pm.energy(Xm)) / (2 * h)
    assert np.max(np.abs(Fp - fd)) < 1e-8 * np.max(np.abs(Fp))
    rng = np.random.default_rng(6)
    V, U = rng.normal(size=X.shape), rng.normal(size=X.shape)
    Hv = pm.hvp(X, V)
    e = [np.linalg.norm(Hv + (pm.forces(X + h * V) - pm.forces(X - h * V)) / (2 * h))
         / np.linalg.norm(Hv) for h in (1e-4, 2e-5)]
    assert e[1] < 1e-7 and e[0] / e[1] > 15.0          # O(h^2) convergence
    assert np.sum(U * Hv) == pytest.approx(np.sum(V * pm.hvp(X, U)), rel=1e-12)


def test_model_pme_total_matches_ewald():
    for bonds in (False, True):
        s = W.with_pme(W.tiny(Q=24, seed=5, bonds=bonds), spacing=0.04, order=8, rtol=1e-12)
        s["epsilon"] = s["epsilon"] * 0.0
        s["bond_k"] = s["bond_k"] * 0.0
        m = Model(s)
        ex = [(int(c // m.Q), int(c % m.Q)) for c in m.excluded]
        assert bool(ex) == bonds
        ew = EW.ewald_energy(s["x"], s["charge"], s["box"], m.beta, m.rc, m.fq, excluded=ex)
        assert m.energy(s["x"]) == pytest.approx(ew["total"], rel=2e-6)


def test_model_pme_forces_and_hvp_against_fd():
    s = W.with_pme(W.tiny(Q=24, seed=5))
    m = Model(s)
    X = s["x"]
    assert len(m.excluded_pairs(X)[0]) > 0
    Fm = m.forces(X)
    h = 1e-6
    fd = np.zeros_like(X)
    for i in range(m.Q):
        for a in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[i, a] += h
            Xm[i, a] -= h
            fd[i, a] = -(m.energy(Xp) - m.energy(Xm)) / (2 * h)
    assert np.max(np.abs(Fm - fd)) < 1e-8 * np.max(np.abs(Fm))
    V = np.random.default_rng(0).normal(size=X.shape)
    Hv = m.hvp(X, V)
    fd = -(m.forces(X + 1e-6 * V) - m.forces(X - 1e-6 * V)) / 2e-6
    assert np.linalg.norm(Hv - fd) < 1e-8 * np.linalg.norm(Hv)
    U = np.random.default_rng(1).normal(size=X.shape)
    assert np.sum(U * Hv) == pytest.approx(np.sum(V * m.hvp(X, U)), rel=1e-10)


def test_real_space_term_reduces_to_coulomb():
    r = np.array([0.15, 0.3, 0.6])
    qq = 2.5
    for beta in (1e-7, 1e-6):
        assert np.allclose(P.ewald_phi(r, qq, beta), qq / r, rtol=1e-6)
        assert np.allclose(P.ewald_d1(r, qq, beta), -qq / r ** 2, rtol=1e-6)
        assert np.allclose(P.ewald_d2(r, qq, beta), 2 * qq / r ** 3, rtol=1e-6)
        # excluded pairs then carry no correction
        assert np.allclose(P.excl_phi(r, qq, beta), 0.0, atol=1e-5)
    beta, h = 3.0, 1e-6
    for fn, d1, d2 in [(P.ewald_phi, P.ewald_d1, P.ewald_d2), (P.excl_phi, P.excl_d1, P.excl_d2)]:
        assert np.allclose(d1(r, qq, beta), (fn(r + h, qq, beta) - fn(r - h, qq, beta)) / (2 * h),
                           rtol=1e-7)
        assert np.allclose(d2(r, qq, beta), (d1(r + h, qq, beta) - d1(r - h, qq, beta)) / (2 * h),
                           rtol=1e-7)
    # erf(beta r)/r -> 2 beta/sqrt(pi) as r -> 0
    assert P.excl_phi(np.array([1e-7]), 1.0, beta)[0] == pytest.approx(
        -2 * beta / math.sqrt(math.pi), rel=1e-9)


def test_with_pme_grid_sizes():
    s = W.with_pme(W.cfg2())
    assert all(k >= L / 0.12 for k, L in zip(s["pme_grid"], s["box"]))
    for k in s["pme_grid"]:
        m = int(k)
        for f in (2, 3, 5, 7):
            while m % f == 0:
                m //= f
        assert m == 1


@pytest.mark.parametrize("name", ["tiny", "water300"])
def test_cell_list_oracle_matches_brute_force_with_pme(name):
    """The C cell-list oracle (Ewald real space and exclusion corrections in C, the mesh
    part from pme.py) equals the numpy brute force for PME systems."""
    from oracle import cl
    base = W.tiny(Q=24, seed=5) if name == "tiny" else W.water_box(300, seed=5, rc=0.6)
    s = W.with_pme(base)
    m, c = Model(s), cl.CellModel(s)
    X = s["x"]
    V = np.random.default_rng(1).normal(size=X.shape)
    assert c.energy(X) == pytest.approx(m.energy(X), rel=1e-12)
    assert np.max(np.abs(c.forces(X) - m.forces(X))) < 1e-12 * np.max(np.abs(m.forces(X)))
    assert np.max(np.abs(c.hvp(X, V) - m.hvp(X, V))) < 1e-12 * np.max(np.abs(m.hvp(X, V)))


def test_pme_path_gradient_matches_finite_differences_of_veff():
    """The exact path gradient of eqs. (5)-(7) with the PME Hessian-vector product is the
    directional derivative of V_eff (eq. 3) with PME forces inside the residuals."""
    from oracle import path as OPth
    s = W.with_pme(W.tiny(Q=20, seed=11))
    m = Model(s)
    R, _, _ = W.random_walk_path(s, 4, 5, sigma=0.003)
    G, _ = OPth.veff_grad(m, R)
    rng = np.random.default_rng(7)
    for _ in range(3):
        u = rng.standard_normal(R.shape)
        u /= np.linalg.norm(u)
        h = 2e-6
        fd = (OPth.veff(m, R + h * u)[0] - OPth.veff(m, R - h * u)[0]) / (2 * h)
        assert abs(fd - np.sum(G * u)) < 2e-6 * np.linalg.norm(G)
