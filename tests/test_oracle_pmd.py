"""Pins of the oracle's path integrator (eq. 4 with the B A O A B splitting) and of its
counter-based normal deviates.

- The Philox4x64-10 implementation reproduces numpy's independent Philox bit generator.
- Box-Muller deviates have the moments and the distribution of a standard normal.
- On a force-free system V_eff is a harmonic chain of springs; velocity Verlet then has
  an exact discrete solution for each normal mode of the chain, which the oracle must
  reproduce to rounding.
- Velocity Verlet is time reversible, and its energy error shrinks as tau^2.
- The Langevin (O) part drives free particles to <M v^2> = kT (1 - c1^(2n)).
"""
import numpy as np
import pytest
from scipy import stats

import workloads as W
from oracle import path as OP
from oracle import philox as PX
from oracle import pmd
from oracle.potential import Model


def free_system(Q, L=20.0, seed=3, mass=None):
    """Q neutral, non-interacting atoms (epsilon = 0, no charges, no bonds): U = 0."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, L, (Q, 3))
    m = rng.uniform(4.0, 30.0, Q) if mass is None else np.full(Q, float(mass))
    return W._system("free", [L, L, L], x, m, np.zeros(Q), np.zeros(Q, int), [0.3], [0.0],
                     np.zeros((0, 2), int), [], [], np.arange(Q), np.zeros(Q, int),
                     rc=0.9, dt=W.DT_PMD, nu=W.NU_PMD)


def test_philox_matches_numpy_bit_generator():
    key = np.array([0x0123456789ABCDEF, 0xFEDCBA9876543210], np.uint64)
    for c0 in (0, 7, 2 ** 64 - 3):
        bg = np.random.Philox(key=key, counter=np.array([c0, 5, 0, 11], np.uint64))
        raw = bg.random_raw(12)
        # numpy advances the counter before each block of four outputs
        ctr = np.array([[(c0 + k) % 2 ** 64, 5, 0, 11] for k in (1, 2, 3)], np.uint64)
        if c0 + 3 >= 2 ** 64:  # carry into the next counter word
            ctr = np.array([[(c0 + k) % 2 ** 64, 5 + (c0 + k >= 2 ** 64), 0, 11]
                            for k in (1, 2, 3)], np.uint64)
        ours = PX.philox4x64_10(ctr, np.tile(key, (3, 1))).ravel()
        assert np.array_equal(ours, raw)


def test_mulhilo_against_python_integers():
    rng = np.random.default_rng(1)
    a = rng.integers(0, 2 ** 63, 200, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    b = rng.integers(0, 2 ** 63, 200, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    hi, lo = PX.mulhilo64(a, b)
    for x, y, h, l in zip(a, b, hi, lo):
        p = int(x) * int(y)
        assert int(h) == p >> 64 and int(l) == p & (2 ** 64 - 1)


def test_uniform_open_interval():
    u = PX.uniform52(np.array([0, 2 ** 64 - 1, 2 ** 63], np.uint64))
    assert u[0] == 2.0 ** -53 and 0.0 < u[0]
    assert u[1] < 1.0 and u[1] == 1.0 - 2.0 ** -53
    assert u[2] == 0.5 + 2.0 ** -53


def test_normals_distribution():
    z = PX.path_normals(seed=99, step=3, N=4, Q=25000).reshape(-1, 3)
    n = z.shape[0]
    for a in range(3):
        assert abs(z[:, a].mean()) < 5.0 / np.sqrt(n)
        assert abs(z[:, a].var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
        assert stats.kstest(z[:, a], "norm").pvalue > 1e-4
    # components and steps are uncorrelated
    c = np.corrcoef(z.T)
    assert np.all(np.abs(c - np.eye(3)) < 5.0 / np.sqrt(n))
    z2 = PX.path_normals(seed=99, step=4, N=4, Q=25000).reshape(-1, 3)
    assert abs(np.mean(z[:, 0] * z2[:, 0])) < 5.0 / np.sqrt(n)


def test_velocity_verlet_harmonic_chain_closed_form():
    """U = 0: V_eff = sum_n K/2 |R^{n+1} - R^n|^2.  With M = m, mode k of the free-end
    chain, u_k(n) = cos(pi k (n - 1/2) / N), has w^2 = (K/m) 4 sin^2(pi k / 2N), and
    velocity Verlet from rest gives q_j = A cos(j theta), cos(theta) = 1 - (w tau)^2/2."""
    N, Q, m = 6, 3, 12.0
    s = free_system(Q, mass=m)
    model = Model(s)
    _, K = OP.coefficients(model)
    tau = 1.0e-3
    for k in (1, 2, 5):
        n = np.arange(1, N + 1)
        u = np.cos(np.pi * k * (n - 0.5) / N)
        w2 = K[0] / m * 4.0 * np.sin(np.pi * k / (2 * N)) ** 2
        theta = np.arccos(1.0 - 0.5 * w2 * tau * tau)
        A = np.array([0.01, -0.02, 0.015])
        R0 = s["x"][None] + u[:, None, None] * A[None, None, :]
        V0 = np.zeros_like(R0)
        steps = 40
        R, V, _, E = pmd.run(model, R0, V0, s["mass"], tau, steps)
        q = np.cos(steps * theta)
        Rx = s["x"][None] + q * u[:, None, None] * A[None, None, :]
        assert np.max(np.abs(R - Rx)) < 1e-12
        vx = -np.sin(steps * theta) * np.sin(theta) / tau
        assert np.max(np.abs(V - vx * u[:, None, None] * A[None, None, :])) < 1e-9
        # discrete energy of the map: K/2 |dR|^2 + M/2 v^2 (1 - (w tau / 2)^2)^-1 ... is
        # conserved only approximately; the spring energy alone follows the closed form
        es = 0.5 * K[0] * np.sum(np.diff(q * u) ** 2) * np.sum(A * A) * Q
        assert E[-1, 0] == pytest.approx(es, rel=1e-9, abs=1e-15)


def test_velocity_verlet_time_reversible():
    s = W.tiny(Q=16, seed=5)
    model = Model(s)
    R0, _, _ = W.random_walk_path(s, 4, 21, sigma=0.002)
    rng = np.random.default_rng(2)
    V0 = rng.normal(0.0, 0.3, R0.shape)
    tau = 2.0e-4
    R1, V1, _, _ = pmd.run(model, R0, V0, s["mass"], tau, 15)
    R2, V2, _, _ = pmd.run(model, R1, -V1, s["mass"], tau, 15)
    assert np.max(np.abs(R2 - R0)) < 1e-10
    assert np.max(np.abs(V2 + V0)) < 1e-7 * np.max(np.abs(V0))


def test_velocity_verlet_energy_error_second_order():
    """Total energy V_eff + kinetic fluctuates by O(tau^2) along a velocity Verlet run."""
    s = W.tiny(Q=16, seed=5)
    model = Model(s)
    R0, _, _ = W.random_walk_path(s, 4, 21, sigma=0.002)
    rng = np.random.default_rng(4)
    V0 = rng.normal(0.0, 0.2, R0.shape)
    T = 0.012
    spread = {}
    for tau in (2.0e-4, 1.0e-4):
        _, _, _, E = pmd.run(model, R0, V0, s["mass"], tau, int(round(T / tau)))
        tot = E.sum(1)
        spread[tau] = tot.max() - tot.min()
    ratio = spread[2.0e-4] / spread[1.0e-4]
    assert 3.0 < ratio < 5.0, ratio


def test_langevin_free_particles_variance():
    """G = 0 (N = 1, U = 0): v_n = c1 v_{n-1} + c2 xi / sqrt(M), so from rest
    <M v^2> per degree of freedom = kT (1 - c1^(2n))."""
    Q = 3000
    s = free_system(Q, L=200.0)
    model = Model(s)
    R0 = s["x"][None].copy()
    V0 = np.zeros_like(R0)
    tau, gamma, kT = 1.0e-3, 250.0, 2.494
    c1 = np.exp(-gamma * tau)
    R = R0
    V = V0
    G = np.zeros_like(R0)
    for n in range(1, 5):
        R, V, G, _, ke, _, _ = pmd.baoab_step(model, R, V, G, s["mass"], tau, gamma, kT,
                                              seed=17, step=n)
        mv2 = s["mass"][:, None] * V[0] ** 2
        expect = kT * (1.0 - c1 ** (2 * n))
        dof = mv2.size
        assert abs(mv2.mean() - expect) < 5.0 * expect * np.sqrt(2.0 / dof)
        assert ke == pytest.approx(0.5 * mv2.sum(), rel=1e-13)
        assert np.max(np.abs(G)) == 0.0


def test_zero_friction_is_velocity_verlet():
    s = W.tiny(Q=16, seed=5)
    model = Model(s)
    R0, _, _ = W.random_walk_path(s, 3, 8, sigma=0.002)
    V0 = np.random.default_rng(6).normal(0.0, 0.2, R0.shape)
    G0, _ = OP.veff_grad(model, R0)
    a = pmd.baoab_step(model, R0, V0, G0, s["mass"], 1e-4, 0.0, 2.5, seed=1, step=0)
    # by hand: kick, drift, gradient, kick
    minv = 1.0 / s["mass"][None, :, None]
    V = V0 - 0.5e-4 * G0 * minv
    R = R0 + 1e-4 * V
    G, ve = OP.veff_grad(model, R)
    V = V - 0.5e-4 * G * minv
    assert np.max(np.abs(a[0] - R)) < 1e-15
    assert np.max(np.abs(a[1] - V)) < 1e-12
    assert a[3] == pytest.approx(ve, rel=1e-14)
