"""GPU parity of the path integrator (pmd_step) against the oracle's B A O A B steps.

Both sides draw the Langevin deviates from their own Philox4x64-10 + Box-Muller
implementation on the same counters, so thermostatted runs are compared step for step.
Tolerances: the FP32 pair terms in the gradient (relative 1e-6 .. 1e-5) are the only
source of difference, so after a few steps positions agree to ~1e-9 nm and velocities
and energies to ~1e-6 relative; the force-free generator check is FP64 throughout.
"""
import numpy as np
import pytest

import workloads as W
from oracle import path as OP
from oracle import philox as PX
from oracle import pmd
from oracle.potential import Model

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mop():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_11962_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(mop):
    return mop.Context()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def cuda(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).cuda()


def say(*a):
    print(*a, flush=True)


def free_system(Q, L=20.0, seed=3):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, L, (Q, 3))
    m = rng.uniform(4.0, 30.0, Q)
    return W._system("free", [L, L, L], x, m, np.zeros(Q), np.zeros(Q, int), [0.3], [0.0],
                     np.zeros((0, 2), int), [], [], np.arange(Q), np.zeros(Q, int),
                     rc=0.9, dt=W.DT_PMD, nu=W.NU_PMD)


def test_generator_matches_oracle(mop, ctx):
    """U = 0 and N = 1: G = 0, so one Langevin step from rest leaves V = c2 xi / sqrt(M)
    and R = R0 + tau/2 V: the device deviates against the oracle's, FP64."""
    Q = 4000
    s = free_system(Q, L=60.0)
    say(f"[pmd generator] Q={Q} N=1")
    plan = mop.Plan(mop.System(ctx, s), 1)
    R = cuda(s["x"][None])
    V = cuda(np.zeros((1, Q, 3)))
    G = cuda(np.zeros((1, Q, 3)))
    tau, gamma, kT, seed = 1e-3, 250.0, 2.494, 0xDEADBEEF12345
    E = mop.pmd_step(plan, R, V, G, tau, 1, gamma, kT, seed, step0=41)
    assert plan.status() == 0
    c1 = np.exp(-gamma * tau)
    c2 = np.sqrt((1 - c1 * c1) * kT)
    xi = PX.path_normals(seed, 41, 1, Q)
    Vx = c2 * xi / np.sqrt(s["mass"])[None, :, None]
    Vg = V.cpu().numpy()
    assert np.max(np.abs(Vg - Vx)) < 1e-13 * np.max(np.abs(Vx))
    assert np.max(np.abs(R.cpu().numpy() - (s["x"][None] + 0.5 * tau * Vx))) < 1e-15 * 60
    Eg = E.cpu().numpy()
    assert Eg[0, 0] == 0.0
    assert Eg[0, 1] == pytest.approx(0.5 * np.sum(s["mass"][None, :, None] * Vx ** 2), rel=1e-12)


@pytest.mark.parametrize("gamma", [0.0, 250.0])
def test_pmd_steps_match_oracle(mop, ctx, gamma):
    s = W.cfg1()
    N, steps, tau, kT, seed = 8, 6, 1e-3, 2.494, 77
    R0, _, _ = W.random_walk_path(s, N, 31, 0.005)
    V0 = np.random.default_rng(9).normal(0.0, 0.3, R0.shape)
    say(f"[pmd] cfg1 N={N} steps={steps} gamma={gamma}")
    plan = mop.Plan(mop.System(ctx, s), N)
    R, V = cuda(R0), cuda(V0)
    G, _ = mop.veff_grad(plan, R)
    E = mop.pmd_step(plan, R, V, G, tau, steps, gamma, kT, seed, step0=5)
    assert plan.status() == 0
    m = Model(s)
    Ro, Vo, Go, Eo = pmd.run(m, R0, V0, s["mass"], tau, steps, gamma, kT, seed, step0=5)
    Rg, Vg, Gg, Eg = (x.cpu().numpy() for x in (R, V, G, E))
    eR = rel(Rg - R0, Ro - R0)
    eV = rel(Vg, Vo)
    eG = rel(Gg, Go)
    say(f"   displacement relL2 {eR:.2e}, V {eV:.2e}, G {eG:.2e}, "
        f"V_eff {np.max(np.abs(Eg[:, 0] - Eo[:, 0]) / np.abs(Eo[:, 0])):.2e}, "
        f"KE {np.max(np.abs(Eg[:, 1] - Eo[:, 1]) / Eo[:, 1]):.2e}")
    assert eR < 1e-6 and eV < 1e-5 and eG < 1e-5
    assert np.allclose(Eg[:, 0], Eo[:, 0], rtol=1e-6)
    assert np.allclose(Eg[:, 1], Eo[:, 1], rtol=1e-6)


def test_pmd_single_bead_and_bad_args(mop, ctx):
    """N = 1 (the polymer is one configuration moving on U) and argument checks."""
    s = W.tiny()
    R0 = s["x"][None].copy()
    V0 = np.random.default_rng(3).normal(0.0, 0.2, R0.shape)
    plan = mop.Plan(mop.System(ctx, s), 2)
    R, V = cuda(R0), cuda(V0)
    G, _ = mop.veff_grad(plan, R)
    E = mop.pmd_step(plan, R, V, G, 2e-4, 4)
    Ro, Vo, _, Eo = pmd.run(Model(s), R0, V0, s["mass"], 2e-4, 4)
    assert rel(R.cpu().numpy() - R0, Ro - R0) < 1e-6
    assert np.allclose(E.cpu().numpy(), Eo, rtol=1e-6)
    for kw in (dict(tau=0.0), dict(tau=-1e-3), dict(tau=1e-3, gamma=-1.0),
               dict(tau=1e-3, kT=-1.0), dict(tau=float("nan"))):
        with pytest.raises(mop.MopError):
            mop.pmd_step(plan, R, V, G, **kw)
    with pytest.raises(mop.MopError):
        mop.pmd_step(plan, R, V, G, 1e-3, nsteps=0)


def test_pmd_nve_energy_conservation(mop, ctx):
    """Velocity Verlet on cfg1 (N = 8): the total energy V_eff + kinetic stays within a
    small fraction of the kinetic-energy fluctuation, and halving tau cuts the spread
    about fourfold (FP32 pair forces add a small noise floor)."""
    s = W.cfg1()
    N = 8
    R0, _, _ = W.random_walk_path(s, N, 31, 0.005)
    V0 = np.random.default_rng(9).normal(0.0, 0.3, R0.shape)
    plan = mop.Plan(mop.System(ctx, s), N)
    spread = {}
    for tau in (2e-4, 1e-4):
        R, V = cuda(R0), cuda(V0)
        G, _ = mop.veff_grad(plan, R)
        E = mop.pmd_step(plan, R, V, G, tau, int(round(0.02 / tau))).cpu().numpy()
        tot = E.sum(1)
        spread[tau] = (tot.max() - tot.min(), E[:, 1].max() - E[:, 1].min())
        say(f"[pmd nve] tau={tau}: total spread {spread[tau][0]:.3e}, kinetic spread "
            f"{spread[tau][1]:.3e}")
        assert spread[tau][0] < 0.05 * spread[tau][1]
    ratio = spread[2e-4][0] / spread[1e-4][0]
    assert 2.5 < ratio < 5.5, ratio
