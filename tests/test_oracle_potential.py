"""Pins of the FP64 oracle's potential, force and Hessian-vector product.

Each test ties the oracle to something other than itself: textbook closed forms of the
pair terms (tests/golden/closed_forms.json), central finite differences, translation
invariance, Hessian symmetry, automatic differentiation of the energy, and brute force
against the independent C cell-list implementation.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle.potential import F_ELEC, Model, reaction_field_constants

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def two_atoms(r, sig=0.3, eps=0.5, q=(0.0, 0.0), L=20.0, rc=6.0, eps_rf=1.0, kb=None, r0=0.1):
    """Two atoms along x in a large periodic box."""
    x = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
    bonds = np.array([[0, 1]]) if kb is not None else np.zeros((0, 2))
    return dict(Q=2, box=np.array([L, L, L]), x=x, mass=np.array([16.0, 16.0]),
                charge=np.array(q, float), type=np.array([0, 0]), sigma=np.array([sig]),
                epsilon=np.array([eps]), bonds=bonds,
                bond_r0=np.array([r0]) if kb is not None else np.zeros(0),
                bond_k=np.array([kb]) if kb is not None else np.zeros(0),
                mol=np.array([0, 1]), molpos=np.array([0, 0]), rc=rc, eps_rf=eps_rf,
                eps_r=1.0, dt=0.001, nu=250.0, kT=2.5)


def axis_curvature(m, x):
    """d^2 U / d x_2^2 along the bond axis, from the oracle's Hessian-vector product."""
    v = np.zeros_like(x)
    v[1, 0] = 1.0
    return m.hvp(x, v)[1, 0]


# --- closed forms -------------------------------------------------------------------

def test_electric_constant_from_codata():
    c = GOLD["codata_2018"]
    f = c["elementary_charge_C"] ** 2 * c["avogadro_per_mol"] / (
        4 * math.pi * c["vacuum_permittivity_F_per_m"] * 1e-9) / 1000.0
    assert abs(f - F_ELEC) / F_ELEC < 1e-8
    assert F_ELEC == GOLD["electric_conversion_kJ_mol_nm_e2"]["value"]


def test_lj_minimum_depth_and_curvature():
    sig, eps = 0.3, 0.5
    g = GOLD["lennard_jones"]
    rm = g["rmin_over_sigma"] * sig
    s = two_atoms(rm, sig, eps)
    m = Model(s)
    # force vanishes at the minimum (the shifted-force correction at 20 sigma is ~1e-7)
    F = m.forces(s["x"])
    assert abs(F[0, 0]) < 1e-6 * eps / sig
    assert np.allclose(F.sum(0), 0.0, atol=1e-15)
    # depth: -eps up to the cutoff shift (|phi(rc)| ~ 4 eps (sig/rc)^6 ~ 3e-8 eps)
    assert abs(m.energy(s["x"]) / eps - g["depth_over_eps"]) < 1e-6
    # curvature along the axis = phi''(r_m)
    k = axis_curvature(m, s["x"])
    assert abs(k * sig ** 2 / eps - g["curvature_sigma2_over_eps"]) < 1e-6 * 57.2
    # off-axis curvature at the minimum is phi'(r)/r = 0 (the pair block is g I + h d d^T)
    v = np.zeros_like(s["x"])
    v[1, 1] = 1.0
    assert abs(m.hvp(s["x"], v)[1, 1]) < 1e-5


def test_coulomb_force_difference_and_curvature():
    # eps_rf = eps_r: no reaction field; the shifted-force constant cancels in differences
    q = (1.0, -1.0)
    r1, r2 = 0.4, 0.7
    m1, m2 = Model(two_atoms(r1, eps=0.0, q=q)), Model(two_atoms(r2, eps=0.0, q=q))
    assert m1.krf == 0.0
    x1, x2 = two_atoms(r1)["x"], two_atoms(r2)["x"]
    f1, f2 = m1.forces(x1)[1, 0], m2.forces(x2)[1, 0]
    # attractive pair: force on atom 2 points to -x with magnitude f/r^2 (plus a constant)
    expect = -F_ELEC * (1.0 / r1 ** 2 - 1.0 / r2 ** 2)
    assert abs((f1 - f2) - expect) < 1e-10 * abs(expect)
    k1 = axis_curvature(m1, x1)
    assert abs(k1 - 2.0 * F_ELEC * q[0] * q[1] / r1 ** 3) < 1e-10 * abs(k1)


def test_reaction_field_limits():
    rc = 1.2
    k_inf, _ = reaction_field_constants(rc, 1e12)
    assert abs(k_inf * rc ** 3 - GOLD["reaction_field"]["k_rf_times_rc3_conducting"]) < 1e-10
    k_eq, c_eq = reaction_field_constants(rc, 1.0)
    assert k_eq == 0.0 and abs(c_eq - 1.0 / rc) < 1e-15
    # the reaction field adds a harmonic term: force difference to plain Coulomb is
    # linear in r with slope -2 f qq k_rf
    q = (0.7, 0.9)
    eps_rf = 78.0
    krf, _ = reaction_field_constants(6.0, eps_rf)
    diffs = []
    for r in (0.5, 1.0, 1.5):
        a = Model(two_atoms(r, eps=0.0, q=q, eps_rf=eps_rf))
        b = Model(two_atoms(r, eps=0.0, q=q, eps_rf=1.0))
        x = two_atoms(r)["x"]
        diffs.append(a.forces(x)[1, 0] - b.forces(x)[1, 0])
    slope1 = (diffs[1] - diffs[0]) / 0.5
    slope2 = (diffs[2] - diffs[1]) / 0.5
    expect = -2.0 * F_ELEC * q[0] * q[1] * krf
    assert abs(slope1 - expect) < 1e-9 * abs(expect)
    assert abs(slope2 - expect) < 1e-9 * abs(expect)


def test_shifted_force_vanishes_at_cutoff():
    s = two_atoms(1.0, sig=0.3, eps=0.6, q=(0.5, -0.3), rc=2.0, eps_rf=78.0)
    m = Model(s)
    rc = m.rc
    i, j = np.array([0]), np.array([1])
    # C^1 at the cutoff: the force vanishes linearly and the energy quadratically in
    # (r_c - r)
    vals = []
    for dlt in (1e-4, 1e-5):
        r = np.array([rc - dlt])
        g, _ = m.pair_gh(r, i, j)
        vals.append((m.pair_phi(r, i, j)[0], g[0] * r[0]))
    (e1, f1), (e2, f2) = vals
    assert abs(f1 / f2 - 10.0) < 1e-3
    assert abs(e1 / e2 - 100.0) < 1e-1
    assert abs(e2) < 1e-8
    # beyond the cutoff nothing interacts
    s2 = two_atoms(rc + 1e-9, sig=0.3, eps=0.6, q=(0.5, -0.3), rc=2.0)
    assert Model(s2).energy(s2["x"]) == 0.0


def test_bond_closed_form():
    kb, r0 = 3.0e5, 0.1
    for r in (0.095, 0.1, 0.108):
        s = two_atoms(r, eps=0.0, kb=kb, r0=r0)
        m = Model(s)
        assert abs(m.energy(s["x"]) - 0.5 * kb * (r - r0) ** 2) < 1e-9
        F = m.forces(s["x"])
        assert abs(F[1, 0] + kb * (r - r0)) < 1e-9          # Hooke's law
        assert abs(axis_curvature(m, s["x"]) - kb) < 1e-6    # d^2/dr^2 = k
        v = np.zeros_like(s["x"])
        v[1, 2] = 1.0                                         # transverse: k (1 - r0/r)
        assert abs(m.hvp(s["x"], v)[1, 2] - kb * (1 - r0 / r)) < 1e-6


def test_exclusions_follow_bond_graph():
    s = W.water_box(30, seed=3, rc=0.3)
    m = Model(s)
    ex = set(m.excluded.tolist())
    Q = s["Q"]
    for w in range(10):
        a, o, b = 3 * w, 3 * w + 1, 3 * w + 2
        assert a * Q + o in ex and o * Q + b in ex and a * Q + b in ex  # 1-2, 1-2, 1-3
    assert len(ex) == 30
    ch = W.cfg3()
    mc = Model(ch)
    Qc = ch["Q"]
    exc = set(mc.excluded.tolist())
    assert 0 * Qc + 1 in exc and 0 * Qc + 2 in exc and 0 * Qc + 3 not in exc  # 1-4 interacts


# --- finite differences, invariances, symmetry --------------------------------------

SYSTEMS = {
    "tiny": lambda: W.tiny(),
    "cfg1": W.cfg1,
    "water": lambda: W.water_box(300, seed=5, rc=0.6),
}


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_force_is_minus_energy_gradient(name):
    s = SYSTEMS[name]()
    m = Model(s)
    x = s["x"]
    rng = np.random.default_rng(11)
    u = rng.standard_normal(x.shape)
    u /= np.linalg.norm(u)
    F = m.forces(x)
    exact = -np.sum(F * u)
    errs = []
    for h in (2e-4, 1e-4):
        fd = (m.energy(x + h * u) - m.energy(x - h * u)) / (2 * h)
        errs.append(abs(fd - exact))
    assert errs[1] < 1e-6 * np.linalg.norm(F) + 1e-9
    assert errs[1] < 0.35 * errs[0] + 1e-9  # second-order convergence


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_translation_invariance(name):
    s = SYSTEMS[name]()
    m = Model(s)
    x = s["x"]
    F = m.forces(x)
    assert np.linalg.norm(F.sum(0)) < 1e-9 * np.linalg.norm(F)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(x.shape)
    HV = m.hvp(x, v)
    assert np.linalg.norm(HV.sum(0)) < 1e-9 * np.linalg.norm(HV)
    t = np.broadcast_to(rng.standard_normal(3), x.shape)
    assert np.linalg.norm(m.hvp(x, t)) < 1e-9 * np.linalg.norm(HV)
    # shifting every atom leaves U and F unchanged
    shift = np.array([0.37, -1.1, 0.52])
    assert abs(m.energy(x + shift) - m.energy(x)) < 1e-9 * abs(m.energy(x))
    assert np.allclose(m.forces(x + shift), F, atol=1e-8 * np.abs(F).max())


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_hessian_symmetry_and_fd(name):
    s = SYSTEMS[name]()
    m = Model(s)
    x = s["x"]
    rng = np.random.default_rng(4)
    u, v = rng.standard_normal(x.shape), rng.standard_normal(x.shape)
    Hu, Hv = m.hvp(x, u), m.hvp(x, v)
    assert abs(np.sum(u * Hv) - np.sum(v * Hu)) < 1e-10 * np.linalg.norm(Hu) * np.linalg.norm(v)
    v /= np.linalg.norm(v)
    Hv = m.hvp(x, v)
    # h below the distance of the nearest cutoff-straddling pair: the second derivative of
    # the shifted-force potential jumps at r_c, so larger steps see an O(h) error
    h = 3e-6
    fd = -(m.forces(x + h * v) - m.forces(x - h * v)) / (2 * h)
    assert np.linalg.norm(fd - Hv) / np.linalg.norm(Hv) < 1e-7


def test_hvp_matches_autograd_of_energy():
    torch = pytest.importorskip("torch")
    s = W.tiny(Q=20, seed=9)
    m = Model(s)
    x0 = s["x"]
    i, j, d = m.pairs(x0)
    shift = d - (x0[j] - x0[i])  # fixed periodic image per pair
    bi, bj, bd = m.bond_vectors(x0)
    bshift = bd - (x0[bj] - x0[bi])
    from oracle.potential import bond_phi

    def energy(X):
        dd = X[j] - X[i] + torch.from_numpy(shift)
        r = torch.sqrt((dd * dd).sum(1))
        e = m.pair_phi(r, i, j).sum()
        bdd = X[bj] - X[bi] + torch.from_numpy(bshift)
        br = torch.sqrt((bdd * bdd).sum(1))
        return e + bond_phi(br, torch.from_numpy(m.bond_r0), torch.from_numpy(m.bond_k)).sum()

    X = torch.tensor(x0, dtype=torch.float64, requires_grad=True)
    E = energy(X)
    assert abs(E.item() - m.energy(x0)) < 1e-10 * abs(E.item())
    (gr,) = torch.autograd.grad(E, X, create_graph=True)
    assert np.allclose(-gr.detach().numpy(), m.forces(x0), rtol=1e-10, atol=1e-10)
    v = np.random.default_rng(5).standard_normal(x0.shape)
    (hv,) = torch.autograd.grad((gr * torch.from_numpy(v)).sum(), X)
    ref = m.hvp(x0, v)
    assert np.linalg.norm(hv.numpy() - ref) < 1e-10 * np.linalg.norm(ref)


# --- brute force vs the C cell-list oracle --------------------------------------------

@pytest.mark.parametrize("name", ["tiny", "cfg1", "water", "cfg2"])
def test_brute_force_equals_cell_list(name, cl_oracle):
    s = W.cfg2() if name == "cfg2" else SYSTEMS[name]()
    m = Model(s)
    cm = cl_oracle.CellModel(s)
    x = s["x"]
    v = np.random.default_rng(6).standard_normal(x.shape)
    U, F, HV = m.energy(x), m.forces(x), m.hvp(x, v)
    U2, F2, HV2 = cm.eval(x, v)
    assert abs(U - U2) < 1e-12 * abs(U)
    assert np.abs(F - F2).max() < 1e-12 * np.abs(F).max()
    assert np.abs(HV - HV2).max() < 1e-12 * np.abs(HV).max()


def test_cell_list_with_many_cells(cl_oracle):
    # 6.2 nm water box, r_c 1.0: 6 cells per axis, unwrapped coordinates far outside the box
    s = W.water_box(3 * 2000, seed=8, rc=1.0)
    m = Model(s)
    cm = cl_oracle.CellModel(s)
    x = s["x"] + np.array([3.0, -2.0, 10.0]) * s["box"]
    U, F = m.energy(x), m.forces(x)
    U2, F2, _ = cm.eval(x)
    assert abs(U - U2) < 1e-12 * abs(U)
    assert np.abs(F - F2).max() < 1e-11 * np.abs(F).max()
