"""Pins of the oracle's effective potential (eq. 3) and its gradient (eqs. 5-7).

The paper prints no numbers for these quantities, so each pin is an identity the
definitions fix: a drift-only Euler path has zero spring energy, a recorded-noise
Euler-Maruyama path has residuals equal to the noise, the gradient matches central
finite differences of V_eff, and the literal effective forces of eqs. (5)-(7) converge
to minus the analytic gradient as the finite-difference parameter shrinks.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import path as P
from oracle.potential import Model

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def em_path(s, m, N, seed, sigma=None, noise=True):
    """Euler-Maruyama discretisation of eq. (1): R^{n+1} = R^n + c F(R^n) + s zeta."""
    c, _ = P.coefficients(m)
    drift = lambda X: c[:, None] * m.forces(X)
    if noise:
        return W.drifted_path(s, N, seed, drift, sigma)
    return W.drifted_path(s, N, seed, drift, 0.0)


def test_k_times_c_is_one_half():
    s = W.tiny()
    c, K = P.coefficients(Model(s))
    assert np.allclose(K * c, GOLD["onsager_machlup"]["K_times_c"], rtol=1e-15)


def test_single_bead_path():
    s = W.tiny()
    m = Model(s)
    R = s["x"][None]
    v, u1, es = P.veff(m, R)
    assert v == u1 == m.energy(s["x"]) and es == 0.0
    G, v2 = P.veff_grad(m, R)
    assert np.allclose(G[0], -m.forces(s["x"]), rtol=0, atol=1e-12)
    assert v2 == v


@pytest.mark.parametrize("mk", [W.tiny, W.cfg1])
def test_drift_only_euler_path_has_no_spring_energy(mk):
    s = mk()
    m = Model(s)
    R, _, _ = em_path(s, m, 6, seed=1, noise=False)
    v, u1, es = P.veff(m, R)
    # each spring term is a rounding residual of R^{n+1} - R^n - c F(R^n)
    assert es < 1e-20 * abs(u1) + 1e-18
    G, _ = P.veff_grad(m, R)
    F1 = m.forces(R[0])
    assert np.abs(G[0] + F1).max() < 1e-9 * np.abs(F1).max()
    assert np.abs(G[1:]).max() < 1e-9 * np.abs(F1).max()


@pytest.mark.parametrize("mk,sigma", [(W.tiny, None), (W.cfg1, 0.005)])
def test_recorded_noise_path_residuals(mk, sigma):
    s = mk()
    m = Model(s)
    R, zeta, sg = em_path(s, m, 5, seed=3, sigma=sigma)
    d, _ = P.residuals(m, R)
    assert np.abs(d - sg[None, :, None] * zeta).max() < 1e-14
    _, K = P.coefficients(m)
    es_closed = 0.5 * np.sum(K[None, :, None] * (sg[None, :, None] * zeta) ** 2)
    _, _, es = P.veff(m, R)
    assert abs(es - es_closed) < 1e-12 * es_closed


def test_brownian_path_equipartition():
    # with s_i^2 = 2 kT c_i, each spring degree of freedom carries kT/2 on average
    s = W.water_box(300, seed=5, rc=0.6)
    m = Model(s)
    R, zeta, sg = em_path(s, m, 9, seed=4)
    _, _, es = P.veff(m, R)
    ndof = 3 * s["Q"] * 8
    mean = es / ndof
    assert abs(mean / (0.5 * s["kT"]) - 1.0) < 5.0 * np.sqrt(2.0 / ndof)


@pytest.mark.parametrize("N", [2, 3, 5])
def test_gradient_matches_finite_differences_of_veff(N):
    s = W.tiny(Q=20, seed=11)
    m = Model(s)
    R, _, _ = em_path(s, m, N, seed=5)
    G, v0 = P.veff_grad(m, R)
    rng = np.random.default_rng(7)
    for _ in range(3):
        u = rng.standard_normal(R.shape)
        u /= np.linalg.norm(u)
        h = 2e-6
        fd = (P.veff(m, R + h * u)[0] - P.veff(m, R - h * u)[0]) / (2 * h)
        assert abs(fd - np.sum(G * u)) < 2e-6 * np.linalg.norm(G)


def test_per_bead_gradient_components_fd():
    # perturb one bead at a time: catches a wrong bead index in the assembly
    s = W.tiny(Q=16, seed=12)
    m = Model(s)
    R, _, _ = em_path(s, m, 4, seed=8)
    G, _ = P.veff_grad(m, R)
    rng = np.random.default_rng(9)
    for n in range(4):
        u = np.zeros_like(R)
        u[n] = rng.standard_normal(R.shape[1:])
        u /= np.linalg.norm(u)
        h = 2e-6
        fd = (P.veff(m, R + h * u)[0] - P.veff(m, R - h * u)[0]) / (2 * h)
        assert abs(fd - np.sum(G[n] * u[n])) < 2e-6 * np.linalg.norm(G[n])


def test_literal_effective_forces_converge_to_minus_gradient():
    s = W.tiny(Q=20, seed=13)
    m = Model(s)
    R, _, _ = em_path(s, m, 5, seed=6)
    G, _ = P.veff_grad(m, R)
    errs = []
    for eps in (2e-2, 1e-2):
        Fe = P.effective_forces_literal(m, R, eps)
        errs.append(np.linalg.norm(Fe + G) / np.linalg.norm(G))
    assert errs[1] < 1e-5
    assert errs[1] < 0.3 * errs[0]  # second order in eps
    # eq. (7): the last bead needs no finite-difference term at all
    Fe = P.effective_forces_literal(m, R, 1e-2)
    assert np.abs(Fe[-1] + G[-1]).max() < 1e-10 * np.abs(G[-1]).max()


def test_fd_gradient_variant_converges():
    s = W.tiny(Q=20, seed=14)
    m = Model(s)
    R, _, _ = em_path(s, m, 4, seed=2)
    G, _ = P.veff_grad(m, R)
    errs = [np.linalg.norm(P.veff_grad_fd(m, R, h) - G) / np.linalg.norm(G) for h in (4e-4, 2e-4)]
    assert errs[1] < 1e-5 and errs[1] < 0.3 * errs[0]


def test_wrapping_beads_into_the_box_changes_nothing():
    s = W.tiny(Q=20, seed=15)
    m = Model(s)
    R, _, _ = em_path(s, m, 4, seed=3)
    shift = np.array([1.0, -2.0, 3.0]) * s["box"]
    Rw = R.copy()
    Rw[1] += shift
    Rw[3] = np.mod(Rw[3], s["box"])
    G, v = P.veff_grad(m, R)
    Gw, vw = P.veff_grad(m, Rw)
    assert abs(v - vw) < 1e-10 * abs(v)
    assert np.abs(G - Gw).max() < 1e-8 * np.abs(G).max()


def test_cell_list_oracle_gives_the_same_path_gradient(cl_oracle):
    s = W.cfg1()
    m = Model(s)
    cm = cl_oracle.CellModel(s)
    R, _, _ = W.random_walk_path(s, 4, 102, 0.005)
    G, v = P.veff_grad(m, R)
    G2, v2 = P.veff_grad(cm, R)
    assert abs(v - v2) < 1e-12 * abs(v)
    assert np.abs(G - G2).max() < 1e-11 * np.abs(G).max()
