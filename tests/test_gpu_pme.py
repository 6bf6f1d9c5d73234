"""GPU parity of particle-mesh Ewald systems: the HIP library (Ewald real-space pair
kernels, fixed-point spreading, rocFFT, FP64 gathers) against the FP64 oracle
(oracle/potential.py with oracle/pme.py).

Tolerances are those of the reaction-field parity tests (relative L2 per bead: forces
1e-5, Hessian-vector products 1e-4, gradient 1e-5; energies 1e-6): the reciprocal part
is FP64 on both sides, so the FP32 real-space pair terms set the error.  A PME energy is
a small difference of large terms (self energy, excluded-pair corrections, real-space
pairs: each about as large as the self energy), and the FP32 pair energies carry an
absolute error of about 1e-8 of those terms, so energies are compared relative to
|U| + |E_self + E_background| rather than |U|.
"""
import numpy as np
import pytest

import workloads as W
from parity_metrics import check
from oracle import ewald as EW
from oracle import mop_bias as MB
from oracle import path as OP
from oracle import pmd
from oracle.potential import Model, min_image

pytestmark = pytest.mark.gpu

TOL_F, TOL_HV, TOL_G, TOL_V = 1e-5, 1e-4, 1e-5, 1e-6


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
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def cuda(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).cuda()


def say(*a):
    print(*a, flush=True)


PME = {
    "tiny": lambda: W.with_pme(W.tiny()),
    "cfg1": lambda: W.with_pme(W.cfg1()),
    "water300": lambda: W.with_pme(W.water_box(300, seed=5, rc=0.6)),
    "water300_p6": lambda: W.with_pme(W.water_box(300, seed=5, rc=0.6), order=6),
    "water300_p8": lambda: W.with_pme(W.water_box(300, seed=5, rc=0.6), order=8, spacing=0.1),
    "cfg2": lambda: W.with_pme(W.cfg2()),
}


@pytest.mark.parametrize("name", list(PME))
def test_pme_bead_forces_and_energy(name, mop, ctx):
    s = PME[name]()
    B = 3
    R, _, _ = W.random_walk_path(s, B, 11)
    plan = mop.Plan(mop.System(ctx, s), B)
    F, U = mop.bead_forces(plan, cuda(R))
    F, U = F.cpu().numpy(), U.cpu().numpy()
    assert plan.status() == 0
    m = Model(s)
    for b in range(B):
        Fo, Uo = m.forces(R[b]), m.energy(R[b])
        ef, eu = rel(F[b], Fo), abs(U[b] - Uo) / (abs(Uo) + abs(m.e_const))
        say(f"[pme {name}] bead {b}: F relL2 {ef:.2e}, U rel {eu:.2e} (U {Uo:.6e})")
        assert ef < TOL_F and eu < TOL_V


@pytest.mark.parametrize("name", list(PME))
def test_pme_bead_hvp(name, mop, ctx):
    s = PME[name]()
    B = 2
    R, _, _ = W.random_walk_path(s, B, 12)
    V = np.random.default_rng(4).normal(0.0, 1e-3, R.shape)
    plan = mop.Plan(mop.System(ctx, s), B)
    H = mop.bead_hvp(plan, cuda(R), cuda(V)).cpu().numpy()
    assert plan.status() == 0
    m = Model(s)
    for b in range(B):
        e = rel(H[b], m.hvp(R[b], V[b]))
        say(f"[pme {name}] bead {b}: Hv relL2 {e:.2e}")
        assert e < TOL_HV


@pytest.mark.parametrize("name,N", [("tiny", 5), ("cfg1", 8), ("water300", 6), ("cfg2", 6)])
def test_pme_veff_grad(name, N, mop, ctx):
    s = PME[name]()
    R, _, _ = W.random_walk_path(s, N, 13, 0.005 if name == "cfg1" else None)
    plan = mop.Plan(mop.System(ctx, s), N)
    G, v = mop.veff_grad(plan, cuda(R))
    G, v = G.cpu().numpy(), float(v[0])
    e3 = mop.veff_energy(plan, cuda(R)).cpu().numpy()
    assert plan.status() == 0
    m = Model(s)
    Go, vo = OP.veff_grad(m, R)
    eg = max(rel(G[n], Go[n]) for n in range(N))
    ev = abs(v - vo) / (abs(vo) + abs(m.e_const))
    say(f"[pme {name}] N={N}: G relL2 (worst bead) {eg:.2e}, V_eff rel {ev:.2e}")
    assert eg < TOL_G
    assert ev < TOL_V
    assert e3[0] == v


@pytest.mark.parametrize("mode", [1, 2])
def test_pme_fd_mode_matches_oracle_fd(mode, mop, ctx):
    s = PME["water300"]()
    N, h = 5, 1e-4
    R, _, _ = W.random_walk_path(s, N, 8)
    plan = mop.Plan(mop.System(ctx, s), N)
    Gfd, _ = mop.veff_grad(plan, cuda(R), mode=mode, fd_h=h)
    assert plan.status() == 0
    m = Model(s)
    Gofd = OP.veff_grad_fd(m, R, h)
    e = rel(Gfd.cpu().numpy(), Gofd)
    say(f"[pme fd] mode {mode}: gpu-FD vs oracle-FD relL2 {e:.2e}")
    assert e < 1e-4


def test_pme_dipole_scale_edge_cases(mop, ctx):
    """bead_hvp with a zero vector gives exactly zero; with a vector 1e6 times larger the
    relative error is unchanged (the fixed-point scale follows max |v|)."""
    s = PME["water300"]()
    R, _, _ = W.random_walk_path(s, 2, 14)
    plan = mop.Plan(mop.System(ctx, s), 2)
    Z = mop.bead_hvp(plan, cuda(R), cuda(np.zeros_like(R))).cpu().numpy()
    assert np.all(Z == 0.0)
    m = Model(s)
    V = np.random.default_rng(5).normal(0.0, 1.0, R.shape)
    for scale in (1e-6, 1.0, 1e3):
        H = mop.bead_hvp(plan, cuda(R), cuda(scale * V)).cpu().numpy()
        e = rel(H[1], m.hvp(R[1], scale * V[1]))
        say(f"[pme] |v| scale {scale:g}: Hv relL2 {e:.2e}")
        assert e < TOL_HV
    assert plan.status() == 0


def test_pme_repeated_calls_bit_identical(mop, ctx):
    """Integer-atomic spreading keeps PME results identical from call to call."""
    s = W.with_pme(W.water_box(1002, seed=9, rc=1.0))
    N = 4
    R, _, _ = W.random_walk_path(s, N, 29)
    plan = mop.Plan(mop.System(ctx, s), N)
    Rt = cuda(R)
    G0, v0 = (x.cpu().numpy() for x in mop.veff_grad(plan, Rt))
    F0, U0 = (x.cpu().numpy() for x in mop.bead_forces(plan, Rt))
    Vt = cuda(np.random.default_rng(3).normal(0.0, 1e-3, R.shape))
    H0 = mop.bead_hvp(plan, Rt, Vt).cpu().numpy()
    for _ in range(3):
        G1, v1 = (x.cpu().numpy() for x in mop.veff_grad(plan, Rt))
        assert np.array_equal(G0, G1) and np.array_equal(v0, v1)
        F1, U1 = (x.cpu().numpy() for x in mop.bead_forces(plan, Rt))
        assert np.array_equal(F0, F1) and np.array_equal(U0, U1)
        assert np.array_equal(H0, mop.bead_hvp(plan, Rt, Vt).cpu().numpy())


def test_pme_one_stream_plan_is_bit_identical(mop, ctx):
    """MOP_PLAN_ONE_STREAM puts the mesh work on the caller's stream (after the pair
    kernels) instead of a second stream beside them, and MOP_PLAN_PERSISTENT launches the
    pair kernels as resident grids over work queues: every result is bit-identical, in
    both gradient modes and through bead_forces / bead_hvp; unknown plan flags are refused."""
    import ctypes as C
    s = W.with_pme(W.water_box(1002, seed=9, rc=1.0))
    N = 4
    R, _, _ = W.random_walk_path(s, N, 31)
    sysm = mop.System(ctx, s)
    plans = [mop.Plan(sysm, N), mop.Plan(sysm, N, one_stream=True),
             mop.Plan(sysm, N, persistent=True)]
    Rt = cuda(R)
    Vt = cuda(np.random.default_rng(4).normal(0.0, 1e-3, R.shape))
    out = []
    for pl in plans:
        G, v = (x.cpu().numpy() for x in mop.veff_grad(pl, Rt))
        Gf, vf = (x.cpu().numpy() for x in mop.veff_grad(pl, Rt, 1, 1e-4))
        F, U = (x.cpu().numpy() for x in mop.bead_forces(pl, Rt))
        H = mop.bead_hvp(pl, Rt, Vt).cpu().numpy()
        assert pl.status() == 0
        out.append((G, v, Gf, vf, F, U, H))
    for a, b, c in zip(*out):
        assert np.array_equal(a, b) and np.array_equal(a, c)
    o = mop._Opts(0.0, 0.0, 0, 8, 0)
    h = C.c_void_p()
    assert mop.lib().mop_plan_create(sysm.h, N, C.byref(o), C.byref(h)) == -1  # MOP_EINVAL


def test_pme_graph_replay_matches_eager(mop, ctx):
    """veff_grad of a PME system (pair kernels, spreading, rocFFT, gathers) captured in
    one graph; every replay, with eager work between replays, equals the eager call."""
    import torch
    s = PME["cfg2"]()
    N = 5
    R, _, _ = W.random_walk_path(s, N, 23)
    plan = mop.Plan(mop.System(ctx, s), N)
    Rt = cuda(R)
    G = torch.empty_like(Rt)
    v = torch.empty(1, dtype=torch.float64, device=Rt.device)
    mop.veff_grad(plan, Rt, 0, 0.0, G, v)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=cs):
        ctx.set_stream()
        mop.veff_grad(plan, Rt, 0, 0.0, G, v)
    ctx.set_stream()
    torch.cuda.synchronize()
    Ge, ve = mop.veff_grad(plan, Rt)
    Ge, ve = Ge.cpu().numpy(), float(ve[0])
    for k in range(3):
        mop.veff_grad(plan, Rt + 1e-3 * (k + 1))
        torch.cuda.synchronize()
        G.zero_()
        g.replay()
        torch.cuda.synchronize()
        same = np.array_equal(G.cpu().numpy(), Ge) and float(v[0]) == ve
        say(f"[pme graph] replay {k}: identical to eager: {same}")
        assert same
    assert plan.status() == 0


def test_pme_biased_path_dynamics(mop, ctx):
    """Langevin path dynamics with the end-to-end bias on a PME system against the
    oracle integrator."""
    s = PME["water300"]()
    N, steps, tau, kT = 5, 3, 1e-3, 2.494
    R0, _, _ = W.random_walk_path(s, N, 31, 0.002)
    V0 = np.random.default_rng(9).normal(0.0, 0.3, R0.shape)
    A, B = np.arange(0, 6), np.arange(150, 159)
    plan = mop.Plan(mop.System(ctx, s), N)
    bias = mop.Bias(plan, A, B, 0.02, 2.0, 4.0, kT, stride=1)
    R, V = cuda(R0), cuda(V0)
    G, _ = mop.veff_grad(plan, R)
    bias.apply(R, G)
    E = mop.pmd_step(plan, R, V, G, tau, steps, 250.0, kT, seed=5, bias=bias).cpu().numpy()
    assert plan.status() == 0
    ob = MB.Bias(A, B, s["mass"], s["box"], 0.02, 2.0, 4.0, kT, stride=1)
    m = Model(s)
    Ro, Vo, _, Eo = pmd.run(m, R0, V0, s["mass"], tau, steps, 250.0, kT, 5, 0, ob)
    e = rel(R.cpu().numpy() - R0, Ro - R0)
    say(f"[pme pmd] displacement relL2 {e:.2e}; V_eff {E[:, 0]} vs {Eo[:, 0]}")
    assert e < 1e-6
    assert np.allclose(E[:, 0], Eo[:, 0], rtol=1e-6, atol=1e-6 * abs(m.e_const))
    assert np.allclose(E[:, 3], Eo[:, 3], rtol=0, atol=1e-8)


def test_pme_parameters_and_restrictions(mop, ctx):
    s = PME["cfg2"]()
    sysm = mop.System(ctx, s)
    grid, beta = sysm.pme_info()
    assert grid == [int(k) for k in s["pme_grid"]]
    assert beta == pytest.approx(EW.beta_from_rtol(s["rc"], 1e-5), rel=1e-12)
    # automatic grid: 2,3,5,7-smooth, >= L/0.12 nm and >= 2 * order
    s2 = dict(s)
    s2.pop("pme_grid")
    g2, _ = mop.System(ctx, s2).pme_info()
    for k, L in zip(g2, s["box"]):
        m = k
        for f in (2, 3, 5, 7):
            while m % f == 0:
                m //= f
        assert m == 1 and k >= L / 0.12 and k >= 8
    with pytest.raises(mop.MopError):
        mop.Plan(sysm, 3, newton3=True)
    plan = mop.Plan(sysm, 3)
    with pytest.raises(mop.MopError):
        mop.Batch([plan], [3])
    rf = mop.System(ctx, W.cfg2())
    with pytest.raises(mop.MopError):
        rf.pme_info()


def _sampled_forces(m, X, idx):
    """Oracle forces on atoms idx only: real-space pairs against every atom, excluded-pair
    corrections, bonds, and the (all-atom) PME reciprocal forces."""
    F = np.zeros((len(idx), 3))
    ex = set(m.excluded.tolist())
    for k, i in enumerate(idx):
        d = min_image(X - X[i], m.box)
        r2 = np.einsum("ak,ak->a", d, d)
        j = np.nonzero((r2 < m.rc ** 2) & (np.arange(m.Q) != i))[0]
        code = np.minimum(i, j) * m.Q + np.maximum(i, j)
        keep = np.array([c not in ex for c in code.tolist()], bool)
        jj = j[keep]
        r = np.sqrt(r2[jj])
        g, _ = m.pair_gh(r, np.full(len(jj), i), jj)
        F[k] = (g[:, None] * d[jj]).sum(0)
        je = j[~keep]
        if len(je):
            from oracle.potential import excl_d1
            re = np.sqrt(r2[je])
            ge = excl_d1(re, m.fq * m.q[i] * m.q[je], m.beta) / re
            F[k] += (ge[:, None] * d[je]).sum(0)
        for b, (bi, bj) in enumerate(m.bonds):
            if i in (bi, bj):
                o = bj if i == bi else bi
                db = min_image(X[o] - X[i], m.box)
                br = float(np.sqrt(db @ db))
                F[k] += m.bond_k[b] * (1.0 - m.bond_r0[b] / br) * db
    return F + m.pme.forces(X)[idx]


def test_pme_cfg4_full_size(mop, ctx):
    """The 150,000-atom membrane-shaped workload with PME (grid at 0.12 nm) in the
    benchmark's launch configuration: the gradient of beads 1 and 16 and the forces of
    bead 1 against the FP64 cell-list oracle (Ewald real space in C, mesh in numpy);
    48 sampled atoms' forces against the brute-force per-atom sum as well."""
    from oracle import cl
    s, R = W.make_config("cfg4")
    s = W.with_pme(s)
    N = R.shape[0]
    plan = mop.Plan(mop.System(ctx, s), N)
    Rt = cuda(R)
    G, v = mop.veff_grad(plan, Rt)
    G = G.cpu().numpy()
    assert plan.status() == 0 and np.isfinite(float(v[0]))
    m = cl.CellModel(s)
    c, K = OP.coefficients(m)
    F0, FN = m.forces(R[0]), m.forces(R[N - 2])
    d0 = min_image(R[1] - R[0], m.box) - c[:, None] * F0
    dN = min_image(R[N - 1] - R[N - 2], m.box) - c[:, None] * FN
    G1 = -F0 - K[:, None] * d0 + 0.5 * m.hvp(R[0], d0)
    say("[pme cfg4] " + check(G[0], G1, TOL_G, "G bead 1"))
    say("[pme cfg4] " + check(G[N - 1], K[:, None] * dN, TOL_G, f"G bead {N}"))
    F, _ = mop.bead_forces(plan, Rt[:1].contiguous(), want_energy=False)
    F = F.cpu().numpy()[0]
    say("[pme cfg4] " + check(F, F0, TOL_F, "bead_forces"))
    idx = np.random.default_rng(7).choice(s["Q"], 48, replace=False)
    es = rel(F[idx], _sampled_forces(Model(s), R[0], idx))
    say(f"[pme cfg4] 48 sampled atoms' forces against the brute-force sum: relL2 {es:.2e}")
    assert es < TOL_F
    HV = mop.bead_hvp(plan, Rt[:1].contiguous(), cuda(d0[None])).cpu().numpy()[0]
    say("[pme cfg4] " + check(HV, m.hvp(R[0], d0), TOL_HV, "bead_hvp (v = d^1)"))
    # the Hessian is symmetric at full size: u . H v = v . H u
    rng = np.random.default_rng(8)
    U = cuda(rng.normal(0.0, 1e-3, (1,) + R.shape[1:]))
    V = cuda(rng.normal(0.0, 1e-3, (1,) + R.shape[1:]))
    HV = mop.bead_hvp(plan, Rt[:1].contiguous(), V).double()
    HU = mop.bead_hvp(plan, Rt[:1].contiguous(), U).double()
    a, b = float((U * HV).sum()), float((V * HU).sum())
    say(f"[pme cfg4] u.Hv {a:.9e}  v.Hu {b:.9e}")
    assert abs(a - b) < 1e-5 * max(abs(a), abs(b))
    assert plan.status() == 0


def test_pme_edge_cases(mop, ctx):
    """A single bead (V_eff = U(R^1), G = -F^1); one charged atom alone in the box (no
    pairs: only its periodic images, the self term and the neutralising background); a
    system with a net charge; coordinates shifted by whole box vectors."""
    # single bead
    s = PME["water300"]()
    R = W.random_walk_path(s, 1, 3)[0]
    plan = mop.Plan(mop.System(ctx, s), 1)
    G, v = mop.veff_grad(plan, cuda(R))
    m = Model(s)
    Fo, Uo = m.forces(R[0]), m.energy(R[0])
    e = rel(-G.cpu().numpy()[0], Fo)
    say(f"[pme edge] N=1: G relL2 {e:.2e}")
    assert e < TOL_F and abs(float(v[0]) - Uo) < TOL_V * (abs(Uo) + abs(m.e_const))
    # one atom
    s1 = W.with_pme(W.tiny(Q=1, charges=False, bonds=False))
    s1["charge"] = np.array([0.7])
    s1["x"] = np.array([[0.31, 0.77, 1.05]])
    plan1 = mop.Plan(mop.System(ctx, s1), 2)
    R1 = np.stack([s1["x"], s1["x"] + 0.01])
    F1, U1 = mop.bead_forces(plan1, cuda(R1))
    m1 = Model(s1)
    for b in range(2):
        Fo1, Uo1 = m1.forces(R1[b]), m1.energy(R1[b])
        say(f"[pme edge] one atom, bead {b}: F {F1.cpu().numpy()[b]} vs {Fo1}, U {float(U1[b]):.9e} vs {Uo1:.9e}")
        assert np.allclose(F1.cpu().numpy()[b], Fo1, rtol=1e-6, atol=1e-9)
        assert float(U1[b]) == pytest.approx(Uo1, rel=1e-10)
    # net charge
    s2 = PME["tiny"]()
    s2["charge"] = s2["charge"] + 0.05
    R2 = W.random_walk_path(s2, 3, 4)[0]
    plan2 = mop.Plan(mop.System(ctx, s2), 3)
    F2, U2 = mop.bead_forces(plan2, cuda(R2))
    m2 = Model(s2)
    for b in range(3):
        ef = rel(F2.cpu().numpy()[b], m2.forces(R2[b]))
        Uo2 = m2.energy(R2[b])
        assert ef < TOL_F and abs(float(U2[b]) - Uo2) < TOL_V * (abs(Uo2) + abs(m2.e_const))
    # unwrapped coordinates
    R3 = W.random_walk_path(s, 3, 5)[0]
    shift = np.random.default_rng(2).integers(-3, 4, R3.shape) * s["box"]
    plan3 = mop.Plan(mop.System(ctx, s), 3)
    Ga, va = mop.veff_grad(plan3, cuda(R3))
    Gb, vb = mop.veff_grad(plan3, cuda(R3 + shift))
    e = rel(Gb.cpu().numpy(), Ga.cpu().numpy())
    say(f"[pme edge] shifted by box vectors: G relL2 {e:.2e}")
    assert e < 1e-7 and abs(float(va[0]) - float(vb[0])) < 1e-9 * abs(float(va[0]))
    for p in (plan, plan1, plan2, plan3):
        assert p.status() == 0
