"""Pins of the oracle's metadynamics-of-paths bias: the end-to-end variable of eq. (8)
and the Gaussian bias on it.

- Centres of mass and the group distance s match hand-placed configurations, also when
  a group straddles the periodic boundary.
- ds/dx matches central finite differences, and sums to zero (translation invariance).
- The Gaussian sum has its closed-form values and slopes at the centre and at one width.
- The bias gradient of a path is the finite-difference gradient of V(S(R)) and touches
  only beads 1 and N.
- Well-tempered heights follow w0 exp(-V/(kT (gamma - 1))); deposits follow the stride.
- With a frozen history, the biased velocity Verlet run conserves V_eff + V_bias + kinetic
  to O(tau^2).
"""
import numpy as np
import pytest

import workloads as W
from oracle import mop_bias as MB
from oracle import pmd
from oracle.potential import Model

BOX = np.array([3.0, 3.2, 3.4])


def test_com_and_distance_hand_placed():
    X = np.zeros((6, 3))
    mass = np.array([1.0, 3.0, 2.0, 2.0, 5.0, 7.0])
    X[0] = [0.2, 0.2, 0.2]
    X[1] = [0.6, 0.2, 0.2]          # A = {0, 1}: COM x = (0.2 + 1.8)/4 = 0.5
    X[2] = [1.5, 1.0, 1.0]
    X[3] = [1.5, 1.4, 1.0]          # B = {2, 3}: COM (1.5, 1.2, 1.0)
    s, e = MB.order_parameter(X, [0, 1], [2, 3], mass, BOX)
    d = np.array([1.0, 1.0, 0.8])
    assert s == pytest.approx(np.linalg.norm(d), rel=1e-14)
    assert np.allclose(e, d / np.linalg.norm(d), atol=1e-15)


def test_group_straddling_the_boundary():
    mass = np.array([2.0, 2.0, 1.0, 1.0])
    X = np.array([[2.95, 1.0, 1.0], [0.05, 1.0, 1.0],     # A straddles x = 0: COM x = 0 (= 3.0)
                  [1.0, 1.0, 1.0], [1.2, 1.0, 1.0]])     # B: COM x = 1.1
    s, _ = MB.order_parameter(X, [0, 1], [2, 3], mass, BOX)
    assert s == pytest.approx(1.1, rel=1e-13)
    # shifting any atom by a box vector changes nothing
    Y = X.copy()
    Y[1, 0] += BOX[0]
    Y[3, 2] -= 2 * BOX[2]
    assert MB.order_parameter(Y, [0, 1], [2, 3], mass, BOX)[0] == pytest.approx(s, rel=1e-13)


def _random_groups(seed, Q=30):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, 1.0, (Q, 3)) * BOX
    mass = rng.uniform(1.0, 16.0, Q)
    A = np.arange(0, 6)
    B = np.arange(10, 19)
    X[A] = X[0] + rng.normal(0, 0.2, (6, 3))
    X[B] = X[10] + rng.normal(0, 0.3, (9, 3))
    return X, mass, A, B


def test_ds_dx_against_finite_differences():
    X, mass, A, B = _random_groups(3)
    g = MB.ds_dx(X, A, B, mass, BOX)
    h = 1e-6
    fd = np.zeros_like(X)
    for i in range(X.shape[0]):
        for a in range(3):
            Xp = X.copy()
            Xm = X.copy()
            Xp[i, a] += h
            Xm[i, a] -= h
            fd[i, a] = (MB.order_parameter(Xp, A, B, mass, BOX)[0]
                        - MB.order_parameter(Xm, A, B, mass, BOX)[0]) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-8
    assert np.max(np.abs(g.sum(0))) < 1e-14
    others = np.setdiff1d(np.arange(X.shape[0]), np.concatenate([A, B]))
    assert np.all(g[others] == 0.0)


def test_gaussian_sum_closed_forms():
    w, sig = 1.7, 0.05
    V, dV = MB.bias(0.3, [0.3], [w], sig)
    assert V == pytest.approx(w, rel=1e-15) and dV == 0.0
    V, dV = MB.bias(0.3 + sig, [0.3], [w], sig)
    assert V == pytest.approx(w * np.exp(-0.5), rel=1e-14)
    assert dV == pytest.approx(-w / sig * np.exp(-0.5), rel=1e-14)
    # two Gaussians symmetric about S: slopes cancel
    V, dV = MB.bias(1.0, [0.9, 1.1], [w, w], sig)
    assert abs(dV) < 1e-12 and V == pytest.approx(2 * w * np.exp(-2.0), rel=1e-14)
    assert MB.bias(0.5, [], [], sig) == (0.0, 0.0)


def test_path_bias_gradient_against_finite_differences():
    s = W.tiny(Q=24, seed=5)
    R, _, _ = W.random_walk_path(s, 4, 9, sigma=0.01)
    A, B = np.arange(0, 4), np.arange(12, 18)
    centers = [0.01, -0.02, 0.005, 0.03]
    heights = [0.8, 1.1, 0.6, 0.9]
    sig = 0.02
    box = s["box"]
    S, V, G = MB.bias_gradient(R, A, B, s["mass"], box, centers, heights, sig)
    assert S == pytest.approx(MB.order_parameter(R[-1], A, B, s["mass"], box)[0]
                              - MB.order_parameter(R[0], A, B, s["mass"], box)[0], rel=1e-14)
    assert np.all(G[1:-1] == 0.0)
    h = 1e-6
    for n in (0, 3):
        for i in list(A[:2]) + list(B[:2]):
            for a in range(3):
                Rp = R.copy()
                Rm = R.copy()
                Rp[n, i, a] += h
                Rm[n, i, a] -= h
                vp = MB.bias(MB.end_to_end(Rp, A, B, s["mass"], box), centers, heights, sig)[0]
                vm = MB.bias(MB.end_to_end(Rm, A, B, s["mass"], box), centers, heights, sig)[0]
                assert G[n, i, a] == pytest.approx((vp - vm) / (2 * h), rel=1e-6, abs=1e-9)


def test_well_tempered_heights_and_stride():
    s = W.tiny(Q=24, seed=5)
    R, _, _ = W.random_walk_path(s, 3, 9, sigma=0.01)
    A, B = np.arange(0, 4), np.arange(12, 18)
    kT, gamma, w0 = 2.5, 6.0, 1.2
    b = MB.Bias(A, B, s["mass"], s["box"], 0.05, w0, gamma, kT, stride=3)
    for step in range(10):
        b.apply(R, step)
    assert len(b.centers) == 4                       # steps 0, 3, 6, 9
    S = MB.end_to_end(R, A, B, s["mass"], s["box"])
    assert np.allclose(b.centers, S, rtol=0, atol=1e-15)
    # the same S each time: V before deposit k is w0 * sum_{j<k} q^j-type closed recursion
    V = 0.0
    for k, w in enumerate(b.heights):
        assert w == pytest.approx(w0 * np.exp(-V / (kT * (gamma - 1.0))), rel=1e-13)
        V += w
    # standard metadynamics keeps the height
    b2 = MB.Bias(A, B, s["mass"], s["box"], 0.05, w0, 0.0, kT, stride=2)
    for step in range(5):
        b2.apply(R, step)
    assert b2.heights == [w0, w0, w0]


def test_biased_nve_conserves_total_energy_with_frozen_history():
    s = W.tiny(Q=16, seed=5)
    model = Model(s)
    R0, _, _ = W.random_walk_path(s, 4, 21, sigma=0.002)
    V0 = np.random.default_rng(4).normal(0.0, 0.2, R0.shape)
    A, B = np.arange(0, 3), np.arange(8, 12)
    S0 = MB.end_to_end(R0, A, B, s["mass"], s["box"])
    spread = {}
    for tau in (2e-4, 1e-4):
        b = MB.Bias(A, B, s["mass"], s["box"], 0.01, 40.0, stride=10 ** 9)
        b.centers, b.heights = [S0 - 0.01, S0 + 0.015], [40.0, 25.0]
        _, _, _, E = pmd.run(model, R0, V0, s["mass"], tau, int(round(0.012 / tau)),
                             step0=1, bias=b)
        tot = E[:, 0] + E[:, 1] + E[:, 2]
        assert np.ptp(E[:, 2]) > 1.0            # the bias does work along the run
        spread[tau] = np.ptp(tot)
    assert 3.0 < spread[2e-4] / spread[1e-4] < 5.0
